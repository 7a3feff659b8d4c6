// Distance-1 coloring (Sec. 5.2) by Jones-Plassmann rounds with hashed
// priorities pi(v) = SplitMix64 finalizer((seed << 32) ^ v) (Steele, Lea,
// Flood 2014).  Priorities are a bijection of v, so every vertex has a
// strict rank; a vertex is coloured once all its higher-priority neighbours
// are, with the smallest colour none of them uses.  The result is therefore
// exactly the greedy colouring in descending priority, for any schedule.
//
// Each vertex keeps the count of its uncoloured higher-priority neighbours;
// colouring a vertex decrements its lower-priority neighbours and those
// reaching zero form the next round's frontier.  The number of rounds is the
// longest priority-descending path, so a round must be short rather than
// wide: one launch per round, and inside it as few dependent memory accesses
// as possible.  One wavefront colours a frontier vertex with a row of up to
// JP_LIGHT entries: every lane loads its (up to four) entries at once, then
// the colours and decrements of all of them, ORs the colours into a 4096-bit
// LDS bitmap of the wave (late vertices of a skewed graph see hundreds of
// colours) and pushes the ready neighbours with one counter update per wave.
// A longer row never gathers its neighbours' colours: every vertex, once
// coloured, ORs its colour into the 4096-bit HBM bitmap of each
// lower-priority long neighbour while decrementing it, so when a long row is
// ready its bitmap already holds the colours of all its higher-priority
// neighbours.  Such a row is cut into JP_CHUNK-entry chunks, one workgroup
// each; every chunk's workgroup reads the row's bitmap, takes the first free
// colour and does its chunk's decrements and ORs, with no merge between the
// workgroups.  The next round is the first to read any colour or bitmap bit
// written in this one (vertices of one round are never adjacent).  Frontier
// sizes live in a device ring indexed by round, so rounds are launched in
// batches without host synchronisation: round r reads slot r, counts the
// next frontier into slot r+1 and clears slot r+2.
#include "lv.h"

#include <vector>

namespace lv {

constexpr int64_t JP_LIGHT = 256;         // rows up to this length: one wavefront per vertex
constexpr int64_t JP_CHUNK = 1024;        // entries of a long row per workgroup
constexpr int JP_BM_WORDS = 64;           // 64 x 64 = 4096 colours in a long row's bitmap
constexpr unsigned JP_LIGHT_BLOCKS = 512; // 2048 waves, grid-stride over the light frontier
constexpr unsigned JP_CHUNK_BLOCKS = 1024;
constexpr int64_t JP_RING = 4;            // slots of 3 counts: light, long vertices, chunks
constexpr int JP_LIGHT_ITEMS = (int)(JP_LIGHT / 64); // entries per lane of a light row
constexpr int JP_CHUNK_ITEMS = (int)(JP_CHUNK / BLOCK); // entries per thread of a chunk
static_assert(JP_LIGHT % 64 == 0 && JP_CHUNK % BLOCK == 0, "whole items per lane");

__device__ __forceinline__ uint64_t jp_priority(uint64_t seed, int64_t v)
{
    uint64_t z = (seed << 32) ^ (uint64_t)v;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// cnt[v] = number of neighbours u != v with pi(u) > pi(v); each thread sums a
// run of consecutive entries per row, rows inside the tile are summed in LDS
__global__ __launch_bounds__(BLOCK) void k_jp_count(Csr g, uint64_t seed, int32_t *cnt)
{
    __shared__ int64_t s_off[ROWCAP + 1];
    __shared__ int64_t s_meta[2];
    __shared__ int32_t s_acc[ROWCAP + 1];
    const int64_t e0 = (int64_t)blockIdx.x * ETILE;
    const int64_t e1 = min(e0 + ETILE, g.nnz) - 1;
    TileRows t = tile_rows(g.off, g.n, e0, e1, s_off, s_meta);
    const int64_t nrows = t.rhi - t.rlo + 1;
    if (t.cached)
        for (int64_t j = threadIdx.x; j < nrows; j += BLOCK) s_acc[j] = 0;
    __syncthreads();
    const int64_t b = e0 + (int64_t)threadIdx.x * EITEMS;
    const int64_t e_end = min(b + EITEMS, e1 + 1);
    if (b <= e1) {
        int64_t row = tile_row(t, g.off, s_off, b);
        int64_t next = tile_off(t, g.off, s_off, row + 1);
        uint64_t prow = jp_priority(seed, row);
        int32_t acc = 0;
        for (int64_t e = b; e < e_end; ++e) {
            while (e >= next) {
                if (acc) {
                    if (t.cached) atomicAdd(&s_acc[row - t.rlo], acc);
                    else atomicAdd(&cnt[row], acc);
                }
                acc = 0;
                ++row;
                next = tile_off(t, g.off, s_off, row + 1);
                if (e >= next) { // empty rows: search instead of stepping through them
                    row = tile_row(t, g.off, s_off, e);
                    next = tile_off(t, g.off, s_off, row + 1);
                }
                prow = jp_priority(seed, row);
            }
            const int32_t u = g.col[e];
            if (u != row && jp_priority(seed, u) > prow) ++acc;
        }
        if (acc) {
            if (t.cached) atomicAdd(&s_acc[row - t.rlo], acc);
            else atomicAdd(&cnt[row], acc);
        }
    }
    __syncthreads();
    if (t.cached)
        for (int64_t j = threadIdx.x; j < nrows; j += BLOCK)
            if (s_acc[j]) atomicAdd(&cnt[t.rlo + j], s_acc[j]);
}

// 1 for the vertices whose rows are longer than JP_LIGHT (their ranks, from a
// scan, index the colour bitmaps)
__global__ __launch_bounds__(BLOCK) void k_jp_long_flags(const int64_t *off, int64_t n, int32_t *flag)
{
    for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * BLOCK)
        flag[v] = off[v + 1] - off[v] > JP_LIGHT ? 1 : 0;
}

// long_id: the rank of a long row, -1 for a light one
__global__ __launch_bounds__(BLOCK) void k_jp_light_ids(const int64_t *off, int64_t n, int32_t *long_id)
{
    for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * BLOCK)
        if (off[v + 1] - off[v] <= JP_LIGHT) long_id[v] = -1;
}

// clears the bitmaps of the *count long rows
__global__ __launch_bounds__(BLOCK) void k_jp_clear_bitmaps(unsigned long long *bm, const int64_t *count)
{
    const int64_t words = *count * JP_BM_WORDS;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < words; i += (int64_t)gridDim.x * BLOCK) bm[i] = 0;
}

// frontier entries carry their rows, so that a round's first dependent read
// is the row itself: a light vertex with its row [b, b + d), and chunk j of
// the long row [rb, rb + d) of v
struct JpItem {
    int64_t b;
    int32_t v, d;
};
struct JpChunk {
    int64_t rb;
    int32_t v, d, j, pad[3];
};
static_assert(sizeof(JpItem) == 16 && sizeof(JpChunk) == 32, "one or two 16-byte loads per entry");

// frontier lists of one round
struct JpLists {
    JpItem *light;
    JpChunk *chunk;
};

// appends the u[j] with ready[j] (rows [ub, ub + ud)) to the next frontier;
// called by all 64 lanes of a wave together.  The light ones take one
// counter update per wave, a long one adds its chunks (counts: light
// vertices, long vertices, chunks)
template <int K>
__device__ __forceinline__ void jp_push(const bool (&ready)[K], const int32_t (&u)[K], const int64_t (&ub)[K],
                                        const int64_t (&ud)[K], const JpLists &out, int32_t *counts)
{
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1;
    unsigned long long m[K];
    int32_t total = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        m[j] = __ballot(ready[j] && ud[j] <= JP_LIGHT);
        total += __popcll(m[j]);
    }
    if (total) {
        int32_t base = 0;
        if (lane == 0) base = atomicAdd(&counts[0], total);
        base = __shfl(base, 0, 64);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if ((m[j] >> lane) & 1) out.light[base + __popcll(m[j] & below)] = JpItem{ub[j], u[j], (int32_t)ud[j]};
            base += __popcll(m[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (ready[j] && ud[j] > JP_LIGHT) {
            atomicAdd(&counts[1], 1);
            const int32_t nch = (int32_t)((ud[j] + JP_CHUNK - 1) / JP_CHUNK);
            const int32_t c0 = atomicAdd(&counts[2], nch);
            for (int32_t q = 0; q < nch; ++q) out.chunk[c0 + q] = JpChunk{ub[j], u[j], (int32_t)ud[j], q, {0, 0, 0}};
        }
}

__global__ __launch_bounds__(BLOCK) void k_jp_start(Csr g, const int32_t *cnt, int32_t *color, JpLists out,
                                                    int32_t *ring)
{
    // the loop runs while any lane of the block has a vertex, so that every
    // wave pushes with all of its lanes
    const int64_t n_up = (g.n + BLOCK - 1) / BLOCK * BLOCK;
    for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n_up; v += (int64_t)gridDim.x * BLOCK) {
        bool ready[1] = {false};
        int32_t u[1] = {(int32_t)v};
        int64_t ub[1] = {0}, ud[1] = {0};
        if (v < g.n) {
            const int64_t b = g.off[v], e = g.off[v + 1];
            const bool alone = (e == b) || (e - b == 1 && g.col[b] == v);
            color[v] = alone ? 0 : -1;
            ready[0] = !alone && cnt[v] == 0;
            ub[0] = b;
            ud[0] = e - b;
        }
        jp_push(ready, u, ub, ud, out, ring);
    }
}

__device__ __forceinline__ unsigned long long wave_or(unsigned long long x)
{
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const unsigned lo = __shfl_xor((unsigned)x, m, 64);
        const unsigned hi = __shfl_xor((unsigned)(x >> 32), m, 64);
        x |= ((unsigned long long)hi << 32) | lo;
    }
    return x;
}

// smallest colour from `base` on that no higher-priority neighbour of v in
// [b, e) uses, by one wavefront in 64-colour windows
__device__ __forceinline__ int32_t jp_wave_mex(const Csr &g, uint64_t seed, int32_t v, uint64_t pv, int64_t b,
                                               int64_t e, const int32_t *color, int32_t base)
{
    const int lane = threadIdx.x & 63;
    for (;; base += 64) {
        unsigned long long used = 0;
        for (int64_t x = b + lane; x < e; x += 64) {
            const int32_t u = g.col[x];
            if (u == v || jp_priority(seed, u) < pv) continue;
            const int32_t cu = color[u] - base;
            if (cu >= 0 && cu < 64) used |= 1ull << cu;
        }
        used = wave_or(used);
        if (used != ~0ull) return base + __ffsll(~used) - 1;
    }
}

// K entries per thread at stride S from x0 (sentinel v past e): the colours
// of the higher-priority neighbours (cu, -1 for the others; read only if HI)
// and the decrements of the lower-priority ones (ready: the decrement reached
// zero, with the row [ub, ub + ud) of such a neighbour; lu: the long-row rank
// of a lower-priority neighbour, -1 for the others).  Loads and atomics of
// the K entries are issued together.
template <int K, int S, bool HI>
__device__ __forceinline__ void jp_entries(const Csr &g, uint64_t seed, int32_t v, uint64_t pv, int64_t x0,
                                           int64_t e, const int32_t *color, int32_t *cnt, const int32_t *long_id,
                                           int32_t (&u)[K], int32_t (&cu)[K], bool (&ready)[K], int64_t (&ub)[K],
                                           int64_t (&ud)[K], int32_t (&lu)[K])
{
    bool hi[K], lo[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int64_t x = x0 + (int64_t)j * S;
        u[j] = x < e ? g.col[x] : v;
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const bool other = u[j] != v;
        hi[j] = other && jp_priority(seed, u[j]) > pv;
        lo[j] = other && !hi[j];
    }
    int32_t old[K];
#pragma unroll
    for (int j = 0; j < K; ++j) cu[j] = (HI && hi[j]) ? color[u[j]] : -1;
#pragma unroll
    for (int j = 0; j < K; ++j) old[j] = lo[j] ? atomicSub(&cnt[u[j]], 1) : 0;
#pragma unroll
    for (int j = 0; j < K; ++j) lu[j] = lo[j] ? long_id[u[j]] : -1;
#pragma unroll
    for (int j = 0; j < K; ++j) ready[j] = lo[j] && old[j] == 1;
#pragma unroll
    for (int j = 0; j < K; ++j) ub[j] = ready[j] ? g.off[u[j]] : 0;
#pragma unroll
    for (int j = 0; j < K; ++j) ud[j] = ready[j] ? g.off[u[j] + 1] - ub[j] : 0;
}

// colour c of a vertex into the bitmaps of its lower-priority long neighbours
template <int K>
__device__ __forceinline__ void jp_mark(unsigned long long *bm, const int32_t (&lu)[K], int32_t c)
{
    if (c >= JP_BM_WORDS * 64) return;
    const unsigned long long bit = 1ull << (c & 63);
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (lu[j] >= 0) atomicOr(&bm[(int64_t)lu[j] * JP_BM_WORDS + (c >> 6)], bit);
}

// one round: light vertices by wavefronts (blocks [0, JP_LIGHT_BLOCKS)),
// chunks of long rows by workgroups (the other blocks).  The first entry of
// a wave or block is read beside the frontier size (cap_*: list capacities;
// an entry past the size is read but not used).
__global__ __launch_bounds__(BLOCK) void k_jp_round(Csr g, uint64_t seed, JpLists in, JpLists out, int32_t *ring,
                                                    int64_t r, int64_t cap_light, int64_t cap_chunk, int32_t *color,
                                                    int32_t *cnt, const int32_t *long_id, unsigned long long *bm)
{
    __shared__ unsigned long long s_wbm[BLOCK / 64][JP_BM_WORDS];
    __shared__ int32_t s_c;
    const int32_t *cur = ring + 3 * (r % JP_RING);
    int32_t *next = ring + 3 * ((r + 1) % JP_RING);
    if (blockIdx.x == 0 && threadIdx.x < 3) ring[3 * ((r + 2) % JP_RING) + threadIdx.x] = 0;
    const int lane = threadIdx.x & 63;
    if (blockIdx.x < JP_LIGHT_BLOCKS) {
        const int64_t f0 = (int64_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
        const int64_t nwaves = (int64_t)JP_LIGHT_BLOCKS * (BLOCK / 64);
        JpItem it = f0 < cap_light ? in.light[f0] : JpItem{0, 0, 0};
        unsigned long long *wbm = s_wbm[threadIdx.x >> 6]; // this wave's bitmap of colours below 4096
        wbm[lane] = 0;
        const int64_t nf = cur[0];
        for (int64_t f = f0; f < nf; f += nwaves) {
            if (f != f0) it = in.light[f];
            const int32_t v = it.v;
            const int64_t b = it.b, e = it.b + it.d;
            const uint64_t pv = jp_priority(seed, v);
            // the row in one pass: colours of the higher-priority neighbours
            // into the wave's LDS bitmap, decrements of the lower-priority
            // ones (their pushes are for the next round, the first to read
            // v's colour), then v's colour into the long ones' bitmaps
            int32_t u[JP_LIGHT_ITEMS], cu[JP_LIGHT_ITEMS], lu[JP_LIGHT_ITEMS];
            bool ready[JP_LIGHT_ITEMS];
            int64_t ub[JP_LIGHT_ITEMS], ud[JP_LIGHT_ITEMS];
            jp_entries<JP_LIGHT_ITEMS, 64, true>(g, seed, v, pv, b + lane, e, color, cnt, long_id, u, cu, ready, ub,
                                                 ud, lu);
#pragma unroll
            for (int j = 0; j < JP_LIGHT_ITEMS; ++j)
                if (cu[j] >= 0 && cu[j] < JP_BM_WORDS * 64) atomicOr(&wbm[cu[j] >> 6], 1ull << (cu[j] & 63));
            jp_push(ready, u, ub, ud, out, next);
            // a wave's LDS operations complete in order: the word read here
            // holds every lane's bits
            const unsigned long long word = wbm[lane];
            wbm[lane] = 0;
            const unsigned long long open = __ballot(word != ~0ull);
            int32_t c;
            if (open) {
                const int l = __ffsll(open) - 1;
                c = l * 64 + __ffsll(~__shfl(word, l, 64)) - 1;
            } else {
                c = jp_wave_mex(g, seed, v, pv, b, e, color, JP_BM_WORDS * 64);
            }
            if (lane == 0) color[v] = c;
            jp_mark(bm, lu, c);
        }
        return;
    }
    const int64_t q0 = blockIdx.x - JP_LIGHT_BLOCKS;
    JpChunk ch = q0 < cap_chunk ? in.chunk[q0] : JpChunk{0, 0, 0, 0, {0, 0, 0}};
    const int64_t nc = cur[2];
    for (int64_t q = q0; q < nc; q += gridDim.x - JP_LIGHT_BLOCKS) {
        if (q != q0) ch = in.chunk[q];
        const int32_t v = ch.v;
        const int64_t rb = ch.rb, re = ch.rb + ch.d;
        const int64_t b = rb + (int64_t)ch.j * JP_CHUNK;
        const int64_t e = min(re, b + JP_CHUNK);
        const uint64_t pv = jp_priority(seed, v);
        if (threadIdx.x < 64) {
            // v's colour: the first free bit of its bitmap, which holds the
            // colours below 4096 of all its higher-priority neighbours; past
            // 4096 by 64-colour windows over the row when all are taken
            static_assert(JP_BM_WORDS == 64, "one bitmap word per lane");
            const unsigned long long word = bm[(int64_t)long_id[v] * JP_BM_WORDS + lane];
            const unsigned long long open = __ballot(word != ~0ull);
            int32_t c;
            if (open) {
                const int l = __ffsll(open) - 1;
                c = l * 64 + __ffsll(~__shfl(word, l, 64)) - 1;
            } else {
                c = jp_wave_mex(g, seed, v, pv, rb, re, color, JP_BM_WORDS * 64);
            }
            if (lane == 0) s_c = c;
        }
        int32_t u[JP_CHUNK_ITEMS], cu[JP_CHUNK_ITEMS], lu[JP_CHUNK_ITEMS];
        bool ready[JP_CHUNK_ITEMS];
        int64_t ub[JP_CHUNK_ITEMS], ud[JP_CHUNK_ITEMS];
        jp_entries<JP_CHUNK_ITEMS, BLOCK, false>(g, seed, v, pv, b + threadIdx.x, e, color, cnt, long_id, u, cu,
                                                 ready, ub, ud, lu);
        jp_push(ready, u, ub, ud, out, next);
        __syncthreads();
        const int32_t c = s_c;
        if (ch.j == 0 && threadIdx.x == 0) color[v] = c;
        jp_mark(bm, lu, c);
        __syncthreads(); // s_c is rewritten by the next chunk
    }
}

__global__ __launch_bounds__(BLOCK) void k_color_max(const int32_t *color, int64_t n, int32_t *out)
{
    int32_t m = -1;
    for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * BLOCK)
        m = max(m, color[v]);
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) m = max(m, __shfl_xor(m, d, 64));
    if ((threadIdx.x & 63) == 0 && m >= 0) atomicMax(out, m);
}

int64_t color_bitmap_words(const Csr &g)
{
    // long rows x bitmap words: a long row has more than JP_LIGHT entries
    return (g.nnz / JP_LIGHT + 1) * JP_BM_WORDS;
}

int64_t color_chunk_pairs(const Csr &g)
{
    // (vertex, chunk) pairs of one frontier: each long row has at most
    // 1 + len / JP_CHUNK chunks
    return g.nnz / JP_CHUNK + g.nnz / JP_LIGHT + 1;
}

int32_t color_jp(const Csr &g, uint64_t seed, const ColorBufs &c, Scratch &s, hipStream_t st)
{
    if (g.n == 0) return 0;
    int32_t *ring = c.counters;
    fill<int32_t>(c.cnt, 0, g.n, st);
    fill<int32_t>(ring, 0, 3 * JP_RING + 1, st);
    unsigned gv = grid_for(g.n, BLOCK * 4);
    if (gv > 4096) gv = 4096;
    k_jp_long_flags<<<gv, BLOCK, 0, st>>>(g.off, g.n, c.long_id);
    scan_i32_to_i32(c.long_id, c.long_id, g.n, s.scalar, s, st);
    k_jp_light_ids<<<gv, BLOCK, 0, st>>>(g.off, g.n, c.long_id);
    k_jp_clear_bitmaps<<<1024, BLOCK, 0, st>>>(c.bm, s.scalar);
    if (g.nnz > 0) k_jp_count<<<grid_for(g.nnz, ETILE), BLOCK, 0, st>>>(g, seed, c.cnt);
    const int64_t cap_chunk = color_chunk_pairs(g);
    JpLists lists[2] = {{(JpItem *)c.light[0], (JpChunk *)c.chunk[0]}, {(JpItem *)c.light[1], (JpChunk *)c.chunk[1]}};
    k_jp_start<<<gv, BLOCK, 0, st>>>(g, c.cnt, c.color, lists[0], ring);
    int64_t r = 0;     // next round to launch
    int64_t batch = 4; // rounds launched per host check, doubled up to 256
    for (;;) {
        for (int64_t i = 0; i < batch; ++i, ++r) {
            const JpLists &in = lists[r & 1], &out = lists[(r + 1) & 1];
            k_jp_round<<<JP_LIGHT_BLOCKS + JP_CHUNK_BLOCKS, BLOCK, 0, st>>>(
                g, seed, in, out, ring, r, g.n, cap_chunk, c.color, c.cnt, c.long_id, c.bm);
        }
        int32_t nf[3] = {0, 0, 0};
        if (hipMemcpyAsync(nf, ring + 3 * (r % JP_RING), 3 * sizeof(int32_t), hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return -1;
        if (nf[0] == 0 && nf[1] == 0 && nf[2] == 0) break;
        if (r > g.n + 256) return -1; // a round colours at least one vertex: cannot happen
        if (batch < 256) batch *= 2;
    }
    int32_t *mx_slot = ring + 3 * JP_RING;
    fill<int32_t>(mx_slot, -1, 1, st);
    k_color_max<<<gv, BLOCK, 0, st>>>(c.color, g.n, mx_slot);
    int32_t mx = -1;
    if (read_back(&mx, mx_slot, st) != hipSuccess) return -1;
    return mx + 1;
}

} // namespace lv

namespace lv {

// ---- balanced colouring ---------------------------------------------------------
// Class-size equalisation of the greedy colouring (Sec. 6.2 finds skewed
// colour classes costly and leaves balanced sets to future work).  With chi
// colours on n vertices the target is gamma = ceil(n / chi).  Over-full
// classes (more than gamma vertices) are taken in ascending colour c; a vertex
// of K_c may go to a colour c' != c that none of its neighbours has and whose
// class holds fewer than gamma vertices (K_c is independent, so this does not
// change while K_c is handled).  In rounds, every waiting vertex of K_c
// proposes its smallest admissible colour (one with none stops waiting); each
// c' takes its proposers in descending priority, at most gamma - |K_c'|; of all
// taken, the first |K_c| - gamma in descending priority move.  K_c is done at
// gamma or after a round that moves nobody.  Every step is a kernel; the host
// keeps the class sizes (chi values) between rounds.

constexpr int BAL_WORDS = 64; // colour bitmap words: up to 4096 colours

__global__ __launch_bounds__(BLOCK) void k_bal_prio_keys(int64_t n, uint64_t seed, uint64_t *keys, int64_t *vals)
{
    for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * BLOCK) {
        keys[v] = ~jp_priority(seed, v); // ascending order = descending priority
        vals[v] = v;
    }
}

__global__ __launch_bounds__(BLOCK) void k_bal_color_keys(int64_t n, const int64_t *vals, const int32_t *color,
                                                          uint64_t *keys, int32_t *size)
{
    for (int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x; p < n; p += (int64_t)gridDim.x * BLOCK) {
        const int32_t c = color[vals[p]];
        keys[p] = (uint64_t)c;
        atomicAdd(&size[c], 1);
    }
}

// one workgroup per waiting vertex of the class: its neighbours' colours into
// an LDS bitmap over the closed colours, then the smallest free colour
__global__ __launch_bounds__(BLOCK) void k_bal_propose(Csr g, const int32_t *list, int64_t count,
                                                       const int32_t *color, const unsigned long long *closed,
                                                       int32_t ncolors, int32_t *waiting, int32_t *prop)
{
    __shared__ unsigned long long s_bm[BAL_WORDS];
    __shared__ int32_t s_first;
    const int words = (ncolors + 63) / 64;
    for (int64_t p = blockIdx.x; p < count; p += gridDim.x) {
        if (!waiting[p]) { // block-uniform
            if (threadIdx.x == 0) prop[p] = -1;
            continue;
        }
        const int32_t v = list[p];
        for (int k = threadIdx.x; k < words; k += BLOCK) s_bm[k] = closed[k];
        if (threadIdx.x == 0) s_first = ncolors;
        __syncthreads();
        for (int64_t e = g.off[v] + threadIdx.x; e < g.off[v + 1]; e += BLOCK) {
            const int32_t u = g.col[e];
            if (u != v) {
                const int32_t cu = color[u];
                atomicOr(&s_bm[cu >> 6], 1ull << (cu & 63));
            }
        }
        __syncthreads();
        for (int k = threadIdx.x; k < words; k += BLOCK) {
            unsigned long long free_bits = ~s_bm[k];
            const int top = ncolors - 64 * k; // colours of this word that exist
            if (top < 64) free_bits &= (1ull << top) - 1;
            if (free_bits) atomicMin(&s_first, 64 * k + __ffsll((long long)free_bits) - 1);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const int32_t d = s_first < ncolors ? s_first : -1;
            prop[p] = d;
            if (d < 0) waiting[p] = 0;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(BLOCK) void k_bal_rank_keys(const int32_t *prop, int64_t count, uint64_t *keys,
                                                         int64_t *vals, int32_t *taken)
{
    for (int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x; p < count; p += (int64_t)gridDim.x * BLOCK) {
        keys[p] = (uint64_t)(prop[p] + 1); // 0: no proposal
        vals[p] = p;
        taken[p] = 0;
    }
}

// proposers grouped by colour (stable: positions ascend = priority descends)
// are taken while their rank is below the colour's room gamma - |K_c'|
__global__ __launch_bounds__(BLOCK) void k_bal_take(const uint64_t *keys, const int64_t *vals, int64_t count,
                                                    const int64_t *first, const int32_t *size, int64_t gamma,
                                                    int32_t *taken)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < count; i += (int64_t)gridDim.x * BLOCK) {
        const uint64_t key = keys[i];
        if (key == 0) continue;
        const int64_t rank = i - first[key];
        if (rank < gamma - size[key - 1]) taken[vals[i]] = 1;
    }
}

// the first `room` taken vertices in priority order move
__global__ __launch_bounds__(BLOCK) void k_bal_apply(const int32_t *list, int64_t count, const int32_t *taken,
                                                     const int32_t *before, int64_t room, const int32_t *prop,
                                                     int32_t c, int32_t *color, int32_t *size, int32_t *waiting)
{
    for (int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x; p < count; p += (int64_t)gridDim.x * BLOCK) {
        if (!taken[p] || before[p] >= room) continue;
        const int32_t d = prop[p];
        color[list[p]] = d;
        atomicAdd(&size[d], 1);
        atomicSub(&size[c], 1);
        waiting[p] = 0;
    }
}

int64_t color_balance(const Csr &g, uint64_t seed, int32_t ncolors, const BalanceBufs &b, Scratch &s, hipStream_t st)
{
    const int64_t n = g.n;
    if (n < 2 || ncolors < 2) return 0;
    if (ncolors > BAL_WORDS * 64) return -2;
    const int64_t gamma = (n + ncolors - 1) / ncolors;
    unsigned gv = grid_for(n, BLOCK * 4);
    if (gv > 65536) gv = 65536;
    // vertices by colour, descending priority within each class
    k_bal_prio_keys<<<gv, BLOCK, 0, st>>>(n, seed, b.keys, b.vals);
    radix_sort(b.keys, b.keys_alt, b.vals, b.vals_alt, n, 64, s, st);
    fill<int32_t>(b.size, 0, ncolors, st);
    k_bal_color_keys<<<gv, BLOCK, 0, st>>>(n, b.vals, b.color, b.keys, b.size);
    int cbits = 1;
    while ((1 << cbits) < ncolors) ++cbits;
    radix_sort(b.keys, b.keys_alt, b.vals, b.vals_alt, n, cbits, s, st);
    narrow_ids(b.vals, b.list, n, st);
    key_offsets(b.keys, n, ncolors, b.first, st);
    std::vector<int64_t> start(ncolors + 1);
    std::vector<int32_t> size(ncolors);
    if (hipMemcpyAsync(start.data(), b.first, (ncolors + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipMemcpyAsync(size.data(), b.size, ncolors * sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return -1;
    int rbits = 1;
    while ((1 << rbits) < ncolors + 1) ++rbits;
    std::vector<unsigned long long> closed(BAL_WORDS);
    int64_t moved_total = 0;
    for (int32_t c = 0; c < ncolors; ++c) {
        if (size[c] <= gamma) continue;
        const int64_t count = size[c]; // K_c has not changed since the grouping
        const int32_t *list = b.list + start[c];
        fill<int32_t>(b.waiting, 1, count, st);
        const unsigned gc = grid_for(count, BLOCK * 4) > 65536 ? 65536 : grid_for(count, BLOCK * 4);
        const unsigned gp = count < 8192 ? (unsigned)count : 8192;
        while (size[c] > gamma) {
            for (auto &w : closed) w = 0;
            for (int32_t d = 0; d < ncolors; ++d)
                if (d == c || size[d] >= gamma) closed[d >> 6] |= 1ull << (d & 63);
            if (hipMemcpyAsync(b.closed, closed.data(), BAL_WORDS * sizeof(unsigned long long), hipMemcpyHostToDevice,
                               st) != hipSuccess)
                return -1;
            k_bal_propose<<<gp, BLOCK, 0, st>>>(g, list, count, b.color, b.closed, ncolors, b.waiting, b.prop);
            k_bal_rank_keys<<<gc, BLOCK, 0, st>>>(b.prop, count, b.keys, b.vals, b.taken);
            radix_sort(b.keys, b.keys_alt, b.vals, b.vals_alt, count, rbits, s, st);
            key_offsets(b.keys, count, ncolors + 1, b.first, st);
            k_bal_take<<<gc, BLOCK, 0, st>>>(b.keys, b.vals, count, b.first, b.size, gamma, b.taken);
            scan_i32_to_i32(b.taken, b.before, count, nullptr, s, st);
            k_bal_apply<<<gc, BLOCK, 0, st>>>(list, count, b.taken, b.before, size[c] - gamma, b.prop, c, b.color,
                                              b.size, b.waiting);
            const int32_t was = size[c];
            if (hipMemcpyAsync(size.data(), b.size, ncolors * sizeof(int32_t), hipMemcpyDeviceToHost, st) !=
                    hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return -1;
            if (size[c] == was) break;
            moved_total += was - size[c];
        }
    }
    return moved_total;
}

} // namespace lv
