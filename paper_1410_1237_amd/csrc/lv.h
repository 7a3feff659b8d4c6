// Internal declarations of the gfx950 Louvain library: device graph views,
// launch helpers and the host-side entry points of each kernel family.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace lv {

typedef __int128 i128;
typedef unsigned __int128 u128;

// weight kinds of a CSR: unit weights (no array), int32 input weights, int64 coarse weights
enum WeightKind : int { W_UNIT = 0, W_I32 = 1, W_I64 = 2 };

struct Csr {
    int64_t n = 0, nnz = 0;
    const int64_t *off = nullptr;
    const int32_t *col = nullptr;
    const void *w = nullptr;
    int wk = W_UNIT;
};

template <int WK> struct WLoad;
template <> struct WLoad<W_UNIT> {
    static __device__ __forceinline__ int64_t at(const void *, int64_t) { return 1; }
};
template <> struct WLoad<W_I32> {
    static __device__ __forceinline__ int64_t at(const void *w, int64_t e) { return ((const int32_t *)w)[e]; }
};
template <> struct WLoad<W_I64> {
    static __device__ __forceinline__ int64_t at(const void *w, int64_t e) { return ((const int64_t *)w)[e]; }
};

constexpr int BLOCK = 256;

inline unsigned grid_for(int64_t items, int64_t per_block)
{
    int64_t g = (items + per_block - 1) / per_block;
    return (unsigned)(g < 1 ? 1 : g);
}

// ---- device helpers -------------------------------------------------------

// smallest power of two >= x (x >= 1)
__host__ __device__ inline int64_t pow2_ceil(int64_t x)
{
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// largest r with off[r] <= e, searching rows [lo, hi) (off ascending)
__device__ __forceinline__ int64_t row_of(const int64_t *off, int64_t lo, int64_t hi, int64_t e)
{
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (off[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// entry-parallel tiles: a block covers ETILE consecutive CSR entries and
// caches the offsets of the rows they span in LDS when they fit
constexpr int EITEMS = 8;
constexpr int ETILE = BLOCK * EITEMS;
constexpr int ROWCAP = 2048;

struct TileRows {
    int64_t rlo, rhi; // rows of the tile's first and last entry
    bool cached;
};

// row_of by all 64 lanes of a wavefront: each step probes 64 offsets evenly
// inside (lo, hi) at once and keeps the bracket between the last probe at
// or below e and the next one, so a search over n rows takes about
// log64(n) dependent loads instead of log2(n).  Same precondition and result
// as row_of; every lane returns the row.
__device__ __forceinline__ int64_t wave_row_of(const int64_t *off, int64_t lo, int64_t hi, int64_t e)
{
    const int lane = threadIdx.x & 63;
    while (hi - lo > 1) {
        const int64_t p = lo + 1 + ((hi - lo - 1) * lane) / 64; // in [lo + 1, hi - 1], nondecreasing in lane
        const unsigned long long m = __ballot(off[p] <= e);    // offsets are sorted: lanes 0..j set
        if (m == 0) {
            hi = __shfl(p, 0, 64);
        } else {
            const int j = 63 - __clzll((long long)m);
            const int64_t pj = __shfl(p, j, 64);
            const int64_t pn = __shfl(p, j < 63 ? j + 1 : 63, 64);
            lo = pj;
            if (j < 63) hi = pn;
        }
    }
    return lo;
}

__device__ __forceinline__ TileRows tile_rows(const int64_t *off, int64_t n, int64_t e0, int64_t e1, int64_t *s_off,
                                              int64_t *s_meta)
{
    if (threadIdx.x < 64) {
        const int64_t lo = wave_row_of(off, 0, n, e0);
        const int64_t hi = wave_row_of(off, lo, n, e1);
        if (threadIdx.x == 0) {
            s_meta[0] = lo;
            s_meta[1] = hi;
        }
    }
    __syncthreads();
    TileRows t;
    t.rlo = s_meta[0];
    t.rhi = s_meta[1];
    const int64_t cnt = t.rhi - t.rlo + 2; // offsets rlo .. rhi+1
    t.cached = cnt <= ROWCAP + 1;
    if (t.cached)
        for (int64_t j = threadIdx.x; j < cnt; j += BLOCK) s_off[j] = off[t.rlo + j];
    __syncthreads();
    return t;
}

// row of entry e inside the tile
__device__ __forceinline__ int64_t tile_row(const TileRows &t, const int64_t *off, const int64_t *s_off, int64_t e)
{
    if (t.cached) {
        int64_t lo = 0, hi = t.rhi - t.rlo + 1;
        while (hi - lo > 1) {
            int64_t mid = (lo + hi) >> 1;
            if (s_off[mid] <= e) lo = mid; else hi = mid;
        }
        return t.rlo + lo;
    }
    return row_of(off, t.rlo, t.rhi + 1, e);
}

__device__ __forceinline__ int64_t tile_off(const TileRows &t, const int64_t *off, const int64_t *s_off, int64_t r)
{
    return t.cached ? s_off[r - t.rlo] : off[r];
}

// ---- primitives (prims.hip) ----------------------------------------------

// Work buffers for scans and sorts; sized by the handle for its largest graph.
struct Scratch {
    int64_t *part = nullptr;   // scan partials
    int64_t part_cap = 0;
    int64_t *scalar = nullptr; // a few device scalars (scan totals etc.)
    int64_t *rep = nullptr;    // RED_REP x 8 replicated counters (rep_add / rep_fold)
};

// Block totals summed into one of RED_REP replicas of up to 8 counters
// (replica r holds counter c at rep[8 r + c], one 64-byte line per replica),
// so that the blocks of a large launch do not all update one word.
constexpr int RED_REP = 64;
__device__ __forceinline__ void rep_add(int64_t *rep, int c, int64_t v)
{
    if (v) atomicAdd((unsigned long long *)&rep[8 * (blockIdx.x % RED_REP) + c], (unsigned long long)v);
}
// out[c] = sum of the replicas of counter c, for c in [0, count)
void rep_fold(const int64_t *rep, int count, int64_t *out, hipStream_t st);
void rep_clear(int64_t *rep, hipStream_t st);

// exclusive scans of n values; *total (device pointer, may be null) gets the sum
void scan_i32_to_i32(const int32_t *in, int32_t *out, int64_t n, int64_t *total, Scratch &s, hipStream_t st);
void scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total, Scratch &s, hipStream_t st);
// head flags of sorted keys (key[e] != key[e-1]) scanned into run ids: out[e] = #heads before e
void scan_heads(const uint64_t *keys, int64_t *out, int64_t n, int64_t *total, Scratch &s, hipStream_t st);
// out[i] = number of j < i with a[j] >= 0
void scan_nonneg(const int32_t *a, int64_t *out, int64_t n, int64_t *total, Scratch &s, hipStream_t st);
// out[i] = sum of the weights w[j] (kind wk) of the j < i with a[j] == tag
void scan_tagged_weights(const int32_t *a, int32_t tag, const void *w, int wk, int64_t *out, int64_t n,
                         int64_t *total, Scratch &s, hipStream_t st);
int64_t scan_partials_needed(int64_t n);

// stable LSD radix sort of (key, value) by the low `bits` bits of key; the
// result ends in keys/vals (the alt buffers are clobbered); vals may be null
void radix_sort(uint64_t *keys, uint64_t *keys_alt, int64_t *vals, int64_t *vals_alt, int64_t n, int bits,
                Scratch &s, hipStream_t st);
int64_t radix_partials_needed(int64_t n);

template <typename T> void fill(T *p, T v, int64_t n, hipStream_t st);

// one device value copied to the host after the work queued before it: the
// first error of the copy or of the wait
template <typename T> hipError_t read_back(T *host, const T *dev, hipStream_t st)
{
    hipError_t e = hipMemcpyAsync(host, dev, sizeof(T), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}
void iota_i32(int32_t *p, int64_t n, hipStream_t st);

// ---- graph kernels (graph.hip) -------------------------------------------

// 0 = valid, else a detail code written to *flag: 1 offsets, 2 column range,
// 3 columns not strictly ascending, 4 weight < 1, 5 asymmetric.  The entry
// checks assume offsets already passed; without `full` only column range.
void validate_csr(const Csr &g, int32_t *flag, hipStream_t st);
void validate_entries(const Csr &g, bool full, int32_t *flag, hipStream_t st);
// k_i = row sums; stats[0] += sum k, stats[1] = max k (atomic), stats[2] += self-loop weights
// range_flag (may be NULL): set to 2 if a column lies outside [0, n)
void degrees(const Csr &g, int64_t *k, int64_t *stats, Scratch &s, hipStream_t st, int32_t *range_flag = nullptr);
// sum of a_c^2 over c in [0, n) into a 128-bit accumulator (out[0] = lo, out[1] = hi)
void sum_squares(const int64_t *a, int64_t n, int64_t *out, Scratch &s, hipStream_t st);
// internal weight of a partition: sum over entries with comm[u] == comm[v]
void internal_weight(const Csr &g, const int32_t *comm, int64_t *out, Scratch &s, hipStream_t st);
// vertex following: map[i] = representative (Sec. 5.3)
void vf_map(const Csr &g, int32_t *map, hipStream_t st);

struct CoarsenBufs {
    int32_t *flag;       // n+1
    int32_t *new_id;     // n+1
    uint64_t *keys, *keys_alt;
    int64_t *vals, *vals_alt;
    int64_t *run;        // nnz (run id of each sorted entry)
    int64_t keys_words;  // capacity of keys (and keys_alt) in 64-bit words
};
// builds the community graph of g under comm into (off_out, col_out, w_out)
// with its weighted degrees k_out and stats = {2m, max degree, self-loop
// total}; returns n' and nnz' (synchronizes); composes orig_map (n_orig entries)
// the same rebuild for a vertex-following map (every community is one kept
// vertex and vertices whose only entry leads to it), by compaction of the
// kept rows instead of a sort; k_in: degrees of g (read before k_out is
// written, so k_out may alias it).  Both return the first error of a copy to
// the host or a wait on the stream (the sizes they read decide the launches
// that follow, so nothing is launched past such an error).
hipError_t coarsen_vf(const Csr &g, const int32_t *map, const int64_t *k_in, int32_t *orig_map, int64_t n_orig,
                      CoarsenBufs &b, int64_t *off_out, int32_t *col_out, int64_t *w_out, int64_t *k_out,
                      int64_t *stats, int64_t *n_new, int64_t *nnz_new, Scratch &s, hipStream_t st);
hipError_t coarsen(const Csr &g, const int32_t *comm, int32_t *orig_map, int64_t n_orig, CoarsenBufs &b,
                   int64_t *off_out, int32_t *col_out, int64_t *w_out, int64_t *k_out, int64_t *stats, int64_t *n_new,
                   int64_t *nnz_new, Scratch &s, hipStream_t st, bool tile_sums);
// tile_sums: sum the (C(u), C(v)) pairs per tile of entries before the sort
// (pays when the partition folds many entries onto few pairs; the output is
// the same either way)
// expands weights of g to int64
void weights_i64(const Csr &g, int64_t *w_out, hipStream_t st);

// ---- sweep (sweep.hip) -----------------------------------------------------

// degree bins: 0 isolated, 1..8 LDS tables (rows up to 2048 entries), 9 and
// 10 hubs (rows above 2048 entries, split across workgroups; bin 9 holds
// rows up to HUB_BIN9_MAX entries, kept apart for the statistics only)
constexpr int NBINS = 11;
constexpr int64_t HUB_BIN9_MAX = 4096;
__host__ __device__ inline int degree_bin(int64_t d)
{
    if (d == 0) return 0;
    if (d <= 4) return 1;
    if (d <= 8) return 2;
    if (d <= 16) return 3;
    if (d <= 32) return 4;
    if (d <= 64) return 5;
    if (d <= 256) return 6;
    if (d <= 1024) return 7;
    if (d <= 2048) return 8;
    if (d <= HUB_BIN9_MAX) return 9;
    return 10;
}

// device accumulators of one sweep launch group; every bin has STAT_REP
// replicas (a block adds to replica blockIdx % STAT_REP) so that the blocks of
// a launch do not all update the same five words; the host sums them
constexpr int STAT_REP = 64;
struct SweepStats {
    int64_t moves;
    int64_t sigma_prev;  // sum over swept vertices of e_{i->C(i)} + w_ii (state read)
    int64_t dsigma;      // sum over movers of 2 (e_{i->c*} - e_{i->C(i)\i})
    int64_t pairs;       // distinct (vertex, community) pairs
    int64_t entries;     // CSR entries gathered
    int64_t pad[3];
};

struct SweepArgs {
    Csr g;
    const int32_t *verts = nullptr; // vertex list of the launch
    int64_t count = 0;              // vertices in the list
    const int32_t *comm_prev = nullptr;
    int32_t *comm_next = nullptr;
    const int64_t *a = nullptr;
    const int32_t *size = nullptr;
    const int64_t *k = nullptr;
    int64_t two_m = 0;
    int singlet = 1;
    int singleton = 0;              // every community is its own vertex (comm_prev[j] == j)
    // (C(j), a_C(j)) of every vertex, C in the low and a in the high 32 bits,
    // or null.  Set only where the totals cannot change during the launch (a
    // plain sweep) and 2m < 2^32 (so a_c and every e_{i->c} fit 32 bits):
    // the rows of bins 1..8 then read a neighbour's community and its total
    // in one gather.
    const uint64_t *cpack = nullptr;
    SweepStats *stats = nullptr;
    // batched graphs (gid == null for a single graph): per-vertex graph id,
    // per-graph 2m, per-graph "sweeping" flag and per-graph stats (8 int64
    // each: moves, sigma_prev, dsigma, pairs, entries)
    const int32_t *gid = nullptr;
    const int64_t *two_m_g = nullptr;
    const int32_t *active_g = nullptr;
    int64_t *gstats = nullptr;
};

// Hub rows (bins 9, 10) run in two passes.  Pass 1: one workgroup per
// HUB_CHUNK-entry chunk sums the chunk per community and writes the distinct
// (community, weight) pairs to the chunk's region of pkey/pval, grouped by
// the community's hash bucket (a hub has P = 2^k buckets, about one per
// HUB_BUCKET entries, at most HUB_PMAX), with the P + 1 bucket boundaries in
// boff.  Pass 2: one workgroup per (hub, bucket) sums the bucket's segments of
// every chunk, evaluates the gains and leaves the bucket's best; one
// wavefront per hub then decides from its buckets' records.  Chunks are half
// the bucket size: on R-MAT the short chunk launches of the colour classes
// finish sooner, and the bucket tables stay as full as before.  Per-position
// prefixes over the sorted vertex
// list: cpre (chunks), bpre (buckets), xpre (boundary entries).
constexpr int HUB_CHUNK = 1024;
constexpr int64_t HUB_BUCKET = 2048;
constexpr int HUB_PMAX = 1024;
__host__ __device__ inline int hub_buckets(int64_t d)
{
    const int64_t p = pow2_ceil((d + HUB_BUCKET - 1) / HUB_BUCKET);
    return (int)(p < HUB_PMAX ? p : HUB_PMAX);
}
// What a hub's pass-1 block (one chunk) and pass-2 block (one bucket) need,
// gathered once per binning so that a block starts from one record instead
// of a chain of dependent lookups (owner position, vertex, prefixes, offsets).
struct HubChunk {
    int32_t v, P;      // the hub and its bucket count
    int64_t beg, end;  // the chunk's entries
    int64_t bo;        // its P + 1 bucket boundaries in boff
    int64_t self_slot; // the hub's first bucket (self-loop slot)
    int64_t pad;
};
struct HubBucket {
    int32_t v, P, b, pad; // the hub, its bucket count, this bucket
    int64_t c0, nch;      // the hub's chunks
    int64_t xo;           // the hub's boundaries in boff
    int64_t pad2;
};

struct HubArgs {
    const int32_t *verts = nullptr; // sorted vertex list (positions are absolute)
    int64_t s = 0, e = 0;           // hub positions [s, e) of this launch group
    const int64_t *cpre = nullptr, *bpre = nullptr, *xpre = nullptr; // n + 1 each
    const struct HubChunk *chunks = nullptr;   // per chunk: what its pass-1 block reads
    const struct HubBucket *buckets = nullptr; // per bucket: what its pass-2 block reads
    int64_t chunk0 = 0, n_chunks = 0;   // cpre[s], cpre[e] - cpre[s]
    int64_t bucket0 = 0, n_buckets = 0; // bpre[s], bpre[e] - bpre[s]
    int32_t *pkey = nullptr;        // HUB_CHUNK pairs per chunk
    void *pval = nullptr;           // uint32 or uint64 per pair (the launch's value width)
    int32_t *boff = nullptr;        // bucket boundaries, P + 1 per chunk
    int64_t *part = nullptr;        // HUB_REC per bucket: best gain (lo, hi), community, e,
                                    // e_A, distinct communities, size of the best community,
                                    // a and size of the hub's own community (state read)
    int64_t *self = nullptr;        // per bucket, used at a hub's first: self-loop weight
                                    // (written by the chunk holding it, cleared by the decision)
};
constexpr int HUB_REC = 10;

// vertices of one degree bin for a fused launch
struct BinRange {
    const int32_t *verts = nullptr;
    int64_t count = 0;
    int64_t block0 = 0;       // first block of the bin (set by the launcher)
    SweepStats *stats = nullptr;
};
struct FusedBins {
    BinRange bins[9];         // index = bin (1..8 used)
    int lanes[9] = {0, 4, 8, 16, 32, 64, 64, 256, 256}; // lanes per vertex (4..64 or 256)
    int64_t hub_block0 = 0;   // first hub pass-1 block of the launch
};
// log2 of the LDS table slots per vertex of bins 0..8 (twice the longest row)
constexpr int kBinShift[9] = {0, 3, 4, 5, 6, 7, 9, 11, 12};
// lanes-per-vertex choices the tuner may take for bins 1..8 (0 ends a list)
constexpr int kLaneChoices[9][4] = {{0}, {4, 8, 0}, {8, 4, 16, 0}, {16, 8, 32, 0}, {32, 16, 64, 0},
                                    {64, 32, 0},     {64, 256, 0}, {256, 0},     {256, 0}};

// out[j] = C(j) | a_C(j) << 32 for the packed gathers (SweepArgs::cpack)
void pack_communities(const int32_t *comm, const int64_t *a, int64_t n, uint64_t *out, hipStream_t st);
// Fused sweep launches (wide = 128-bit gains, narrow = hub sums fit 32
// bits); each returns false when it had nothing to launch.  small: bins 1..5;
// large: bins 6..7 plus hub pass 1; bin8: bin 8 alone; all: bins 1..8 plus
// hub pass 1 (small groups); then hub pass 2 and, in a launch of its own, the
// hub decisions (stats in a.stats).
bool sweep_small(const SweepArgs &a, FusedBins f, bool wide, hipStream_t st);
bool sweep_large(const SweepArgs &a, FusedBins f, const HubArgs &h, bool wide, bool narrow, hipStream_t st);
bool sweep_bin8(const SweepArgs &a, const FusedBins &f, bool wide, bool narrow, hipStream_t st);
bool sweep_all(const SweepArgs &a, FusedBins f, const HubArgs &h, bool wide, bool narrow, hipStream_t st);
// decide = false leaves the hub decisions to commit_hubs
bool sweep_hub_agg(const SweepArgs &a, const HubArgs &h, bool wide, bool narrow, bool decide, hipStream_t st);
// commit of a colour class (positions [pos0, pos0 + count) of the sorted
// vertex list) that first makes the decisions of the class's hubs
void commit_hubs(const SweepArgs &a, const HubArgs &h, const int32_t *list, int64_t pos0, int64_t count, bool wide,
                 hipStream_t st);
// per-vertex degree bin keys for sorting: key = (group << 4) | bin, val = vertex
// (batched form: vertices of graphs with active[gid[v]] == 0 go to bin 0,
// which is never swept)
void bin_keys(const Csr &g, const int32_t *group, uint64_t *keys, int64_t *vals, hipStream_t st,
              const int32_t *gid = nullptr, const int32_t *active = nullptr);
// off[key] = first index of the sorted keys with key >= key, key in [0, nkeys]
void key_offsets(const uint64_t *keys, int64_t n, int64_t nkeys, int64_t *off, hipStream_t st);
// vertex ids from sorted bin values (int64 -> int32)
void narrow_ids(const int64_t *vals, int32_t *out, int64_t n, hipStream_t st);
// per position of verts: cpre, bpre, xpre = prefixes of hub chunks, buckets
// and bucket-boundary entries (n + 1 each; the totals land at index count)
void hub_prefix(const Csr &g, const int32_t *verts, int64_t count, int64_t *cpre, int64_t *bpre, int64_t *xpre,
                Scratch &s, hipStream_t st);
// the chunk and bucket records of the hubs among positions [0, count) of the
// sorted vertex list verts
void hub_owners(const int32_t *verts, const int64_t *off, const int64_t *cpre, const int64_t *bpre,
                const int64_t *xpre, int64_t count, HubChunk *chunks, HubBucket *buckets,
                hipStream_t st);
void gather_i64(const int64_t *src, const int64_t *idx, int64_t n, int64_t *out, hipStream_t st);
// community degree/size updates for movers in the list (or all vertices if verts == null)
void commit(const int32_t *verts, int64_t count, int32_t *comm_prev, const int32_t *comm_next,
            const int64_t *k, int64_t *a, int32_t *size, hipStream_t st);
void clear_stats(SweepStats *s, int count, hipStream_t st);

// ---- batched graphs (batch.hip) ------------------------------------------------
void graph_ids(const int64_t *goff, int32_t ng, int64_t n, int32_t *gid, hipStream_t st);
// flag := 6 when an entry joins two different graphs
void cross_edges(const Csr &g, const int32_t *gid, int32_t *flag, hipStream_t st);
// out[4g..4g+3]: sum x, sum x^2 (lo, hi), self-loop weight (if with_self)
void graph_sums(const Csr &g, bool with_self, const int64_t *x, const int32_t *gid, int32_t ng, int64_t *out,
                hipStream_t st);
// chain-compressing vertex following, one round: map[i] = the vertex i
// follows (itself if none); *moved (device) = vertices that follow another.
// gid/g_two_m (may be null): per-graph 2m of a batch
void vf_chain_map(const Csr &g, const int64_t *k, int64_t two_m, const int32_t *gid, const int64_t *g_two_m,
                  int32_t *map, int64_t *moved, Scratch &s, hipStream_t st);
// per graph: mode 1 commits (keeping the replaced partition in comm_save),
// 2 restores comm_save, 0 drops the proposals
void commit_graphs(int64_t n, int32_t *comm_prev, int32_t *comm_next, int32_t *comm_save, const int64_t *k,
                   int64_t *a, int32_t *size, const int32_t *gid, const int32_t *mode, hipStream_t st);
void new_graph_offsets(const int64_t *goff, int32_t ng, int64_t n, const int32_t *new_id, int64_t total,
                       int64_t *new_goff, hipStream_t st);
void local_labels(const int32_t *orig_map, const int32_t *gid0, int64_t n0, const int64_t *goff, int32_t *labels,
                  hipStream_t st);
// per-graph arrays copied side by side -> union CSR (adds each graph's first
// entry to its offsets and its first vertex to its columns)
void batch_fixup(int64_t *off, int64_t n, int32_t *col, int64_t nnz, const int64_t *goff, const int64_t *eoff,
                 int32_t ng, hipStream_t st);

// ---- coloring (color.hip) ---------------------------------------------------

// device buffers of a colouring (n = vertices of the graph)
struct ColorBufs {
    int32_t *color;          // n: the colours
    int32_t *cnt;            // n: uncoloured higher-priority neighbours
    int32_t *long_id;        // n: rank among the rows longer than the light limit
    int32_t *counters;       // 16: frontier-size ring and the colour maximum
    void *light[2];          // n entries of 16 bytes each: light frontier lists (ping-pong)
    void *chunk[2];          // color_chunk_pairs entries of 32 bytes each: chunks of long rows
    unsigned long long *bm;  // color_bitmap_words: colour bitmaps of long rows
};
int64_t color_bitmap_words(const Csr &g);
int64_t color_chunk_pairs(const Csr &g);
// Jones-Plassmann coloring; returns the number of colors (synchronizes)
// returns the colour count, or -1 if a copy or wait of the stream failed
int32_t color_jp(const Csr &g, uint64_t seed, const ColorBufs &c, Scratch &s, hipStream_t st);

// buffers of the balanced colouring: color (in/out); list, waiting, prop,
// taken, before int32[n]; size int32[ncolors]; closed u64[64]; the radix
// sort's keys/vals pairs (n each); first int64[ncolors + 2]
struct BalanceBufs {
    int32_t *color, *list, *waiting, *prop, *taken, *before, *size;
    unsigned long long *closed;
    uint64_t *keys, *keys_alt;
    int64_t *vals, *vals_alt, *first;
};
// balances the class sizes of a greedy colouring (color.hip); returns the
// vertices moved, -1 if a copy or wait of the stream failed, -2 if ncolors
// exceeds 4096
int64_t color_balance(const Csr &g, uint64_t seed, int32_t ncolors, const BalanceBufs &b, Scratch &s,
                      hipStream_t st);

} // namespace lv
