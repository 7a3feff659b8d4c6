// Host runtime and C ABI of liblouvain.so: the handle (device arena, stream,
// phase state), the phase driver of the paper's parallel algorithm
// (Sec. 5.4: vertex following, coloring, phases of synchronous sweeps,
// rebuild) with the coloring schedule and thresholds of Sec. 6.1, and exact
// 128-bit host arithmetic for modularity and thresholds.
#include "louvain.h"
#include "lv.h"

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <cstdlib>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

using lv::i128;
using lv::u128;

// ---------------------------------------------------------------------------
// process-wide caching pool of device buffers (reused across handles of equal
// sizes so that repeated ingest/run/destroy cycles do not re-allocate)
// ---------------------------------------------------------------------------
namespace {

struct Pool {
    std::mutex mu;
    std::map<std::pair<int, size_t>, std::vector<void *>> free_; // (device, size class) -> blocks
    size_t cached = 0;
    static constexpr size_t CAP = (size_t)96 << 30;

    // size classes: 8 per power of two (at most 12.5 % rounding), 256-byte
    // minimum, so that buffers of nearby sizes are reused
    static size_t size_class(size_t bytes)
    {
        if (bytes <= 256) return 256;
        const int lg = 63 - __builtin_clzll((unsigned long long)(bytes - 1)); // bytes in (2^lg, 2^(lg+1)]
        const size_t step = (size_t)1 << (lg - 3);                            // lg >= 8 here
        return (bytes + step - 1) / step * step;
    }

    hipError_t get(void **p, size_t bytes, int dev)
    {
        const size_t cls = size_class(bytes);
        {
            std::lock_guard<std::mutex> lk(mu);
            auto it = free_.find({dev, cls});
            if (it != free_.end() && !it->second.empty()) {
                *p = it->second.back();
                it->second.pop_back();
                cached -= cls;
                return hipSuccess;
            }
        }
        hipError_t e = hipMalloc(p, cls);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            trim(dev);
            e = hipMalloc(p, cls);
        }
        return e;
    }
    void put(void *p, size_t bytes, int dev)
    {
        if (!p) return;
        const size_t cls = size_class(bytes);
        std::lock_guard<std::mutex> lk(mu);
        if (cached + cls > CAP) {
            (void)hipFree(p);
            return;
        }
        free_[{dev, cls}].push_back(p);
        cached += cls;
    }
    void trim(int dev)
    {
        std::lock_guard<std::mutex> lk(mu);
        for (auto &kv : free_) {
            if (kv.first.first != dev) continue;
            for (void *p : kv.second) {
                (void)hipFree(p);
                cached -= kv.first.second;
            }
            kv.second.clear();
        }
    }
};
Pool &pool()
{
    static Pool *p = new Pool(); // never destroyed: buffers live until process end
    return *p;
}

std::string g_init_error;

// ---- exact host arithmetic ---------------------------------------------------
u128 mag(i128 x) { return x < 0 ? (u128)0 - (u128)x : (u128)x; }

// x*p < y*q with x, y < 2^127 and p, q < 2^64, by 64-bit limbs
bool prod_less(u128 x, uint64_t p, u128 y, uint64_t q)
{
    auto mul = [](u128 a, uint64_t b, uint64_t out[3]) {
        const u128 lo = (u128)(uint64_t)a * b;
        const u128 hi = (u128)(uint64_t)(a >> 64) * b + (lo >> 64);
        out[0] = (uint64_t)lo;
        out[1] = (uint64_t)hi;
        out[2] = (uint64_t)(hi >> 64);
    };
    uint64_t a[3], b[3];
    mul(x, p, a);
    mul(y, q, b);
    for (int t = 2; t >= 0; --t)
        if (a[t] != b[t]) return a[t] < b[t];
    return false;
}

// net gain below theta: (now - before) < theta * ref, ref = |before| (relative) or D (absolute)
bool below_threshold(i128 now, i128 before, i128 D, louvain_ratio th, int mode)
{
    if (now < before) return true;
    const u128 gain = (u128)(now - before);
    const u128 ref = mode == 0 ? mag(before) : (u128)D;
    return prod_less(gain, (uint64_t)th.den, ref, (uint64_t)th.num);
}

// correctly rounded (ties to even) double of N / D, 0 < D, |N| <= D
double exact_ratio(i128 N, i128 D)
{
    if (N == 0) return 0.0;
    const bool neg = N < 0;
    u128 num = mag(N);
    const u128 den = (u128)D;
    // scale num by 2^s (s <= 0) so that den <= num < 2 den; |N| <= D keeps num < 2^127
    int s = 0;
    while (num < den) {
        num <<= 1;
        --s;
    }
    // 53 significant bits + guard bit by restoring division
    uint64_t q = 0;
    u128 r = num;
    for (int b = 0; b < 54; ++b) {
        q <<= 1;
        if (r >= den) {
            q |= 1;
            r -= den;
        }
        r <<= 1;
    }
    // q holds 54 bits: value = q * 2^(s - 53)
    const bool guard = q & 1;
    q >>= 1;
    int e = s - 52;
    if (guard && (r != 0 || (q & 1))) {
        ++q;
        if (q == (1ull << 53)) {
            q >>= 1;
            ++e;
        }
    }
    double v = std::ldexp((double)q, e);
    return neg ? -v : v;
}

louvain_i128 to_abi(i128 v)
{
    louvain_i128 r;
    r.lo = (uint64_t)(u128)v;
    r.hi = (int64_t)(v >> 64);
    return r;
}

double ms_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

int bits_for(int64_t n)
{
    int b = 1;
    while (((int64_t)1 << b) < n) ++b;
    return b;
}

struct ProfRec {
    const char *name;
    int64_t launches = 0;
    double ms = 0, bytes = 0, entries = 0;
};

} // namespace

// ---------------------------------------------------------------------------
// the handle
// ---------------------------------------------------------------------------
struct louvain_graph_s {
    hipStream_t st = nullptr;
    int dev = 0;
    std::string err;
    bool poisoned = false;
    std::vector<std::pair<void *, size_t>> owned;
    // set for the allocation-free entry point: buffers are carved in order
    // from this device range instead of the pool (count_only: sizes summed,
    // nothing carved, no device work)
    char *arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    bool count_only = false;

    // input graph (level 0)
    int64_t n0 = 0, nnz0 = 0, two_m = 0, kmax0 = 0, self0 = 0;
    int64_t *off0 = nullptr, *k0 = nullptr;
    int32_t *col0 = nullptr, *w0 = nullptr;
    // coarse graph buffers (ping-pong)
    int64_t *off_b[2] = {nullptr, nullptr}, *w_b[2] = {nullptr, nullptr};
    int32_t *col_b[2] = {nullptr, nullptr};
    int cur_buf = -1; // -1: level 0
    int level = 0;
    lv::Csr cur;
    int64_t kmax = 0, self = 0;

    // phase state
    int64_t *k = nullptr, *a = nullptr;
    int32_t *comm_prev = nullptr, *comm_next = nullptr, *size = nullptr, *orig_map = nullptr;
    int32_t *comm_save = nullptr; // partition before the last committed iteration (undo of a loss)
    int64_t sigma_in = 0; // internal weight of the current partition (step API)
    int64_t swept_entries = 0; // entries gathered by every sweep of the current run
    int64_t lookahead_entries = 0; // of those, by look-ahead sweeps whose moves were discarded

    // coloring
    int32_t *color = nullptr, *jp_cnt = nullptr, *counters = nullptr;
    int64_t *jp_light = nullptr;            // two light frontier lists of n 16-byte entries
    int64_t *jp_chunk = nullptr;            // two chunk lists of 32-byte entries
    uint64_t *jp_bm = nullptr;              // colour bitmaps of long rows (cleared by each colouring)
    unsigned long long *bal_closed = nullptr; // closed-colour bitmap of the balanced colouring (64 words)
    int64_t jp_chunk_cap = 0, jp_bm_cap = 0;
    int64_t keys_words = 0;                 // capacity of keys / keys_alt
    int tile_sums_mode = -1;                // rebuild pair sums: -1 by the pair count, 0 never, 1 always
    int32_t num_colors = 0;
    bool colored = false;
    bool singleton = false; // state is the singleton partition (no commit since init_state)
    int lanes[9] = {0, 4, 8, 16, 32, 64, 64, 256, 256}; // lanes per vertex of bins 1..8 (tuned)
    bool tune = true;       // LOUVAIN_AUTOTUNE=0 keeps the default lanes

    // binning
    uint64_t *keys = nullptr, *keys_alt = nullptr;
    int64_t *vals = nullptr, *vals_alt = nullptr, *run = nullptr;
    int32_t *bin_verts = nullptr, *bin_hist = nullptr;
    int64_t bin_hist_cap = 0;
    std::vector<int64_t> bin_off; // (group*16 + bin) -> start in bin_verts; size 16*groups + 1
    int bin_groups = 0;
    bool bins_valid = false;
    bool bins_colored = false;
    int64_t *bin_offd = nullptr;  // device copy of bin_off (capacity bin_hist_cap + 1)
    int64_t *cpre = nullptr, *bpre = nullptr, *xpre = nullptr; // hub prefixes per bin-list position
    int32_t *pkey = nullptr, *boff = nullptr;
    uint64_t *pval = nullptr;
    int64_t *hpart = nullptr, *hself = nullptr;
    lv::HubChunk *chunk_rec = nullptr;
    lv::HubBucket *bucket_rec = nullptr;
    int64_t pcap = 0, xcap = 0, qcap = 0;   // pairs, bucket boundaries, buckets allocated
    std::vector<lv::HubArgs> hub_groups;    // per group (e <= s when the group has no hub)

    // coarsening
    int32_t *flag = nullptr, *new_id = nullptr;
    lv::Scratch scratch;
    lv::SweepStats *stats = nullptr; // NBINS slots
    int64_t *dscal = nullptr;        // 16 device scalars
    int32_t *vflag = nullptr;

    // batched graphs: set while a batch runs on this union graph
    const int32_t *b_gid = nullptr;
    const int64_t *b_two_m = nullptr;
    const int32_t *b_active = nullptr;
    int64_t *b_gstats = nullptr;

    // results
    std::vector<louvain_phase_stats> phases;
    std::vector<louvain_iter_stats> iters;

    // launch sequences captured as HIP graphs and replayed while the bins and
    // buffers they were captured on stay the same (epoch)
    struct Stage {
        hipGraphExec_t exec = nullptr;
        uint64_t epoch = ~0ull;
    };
    hipStream_t gst = nullptr;           // private stream: graphs are captured on and launched from it
    hipEvent_t gev[2] = {nullptr, nullptr};
    bool graphs_ok = true;               // cleared if a capture is refused (then stages run eagerly)
    bool graph_colored = false;          // capture the colour classes too (measured slower on MI355X)
    uint64_t epoch = 0;
    Stage stage_colored, stage_batch;

    // profiling
    bool prof = false;
    std::vector<ProfRec> recs;
    struct Pending {
        hipEvent_t a, b;
        int rec;
        double bytes, entries;
        int stat_slot;
        bool from_stats;
        bool singleton; // a sweep from the singleton partition (no community gather)
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
};

namespace {

typedef louvain_graph_s G;

louvain_status fail(G *g, louvain_status s, const std::string &msg)
{
    if (g) g->err = msg;
    else g_init_error = msg;
    return s;
}

louvain_status hip_fail(G *g, hipError_t e, const char *where)
{
    g->poisoned = true;
    return fail(g, LOUVAIN_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(g, call)                                                                                        \
    do {                                                                                                       \
        hipError_t e_ = (call);                                                                                \
        if (e_ != hipSuccess) return hip_fail(g, e_, #call);                                                   \
    } while (0)

template <typename T> louvain_status alloc(G *g, T **p, int64_t count)
{
    const size_t bytes = (size_t)(count > 0 ? count : 1) * sizeof(T);
    if (g->arena || g->count_only) {
        const size_t need = (bytes + 255) & ~(size_t)255;
        if (g->count_only) {
            g->arena_used += need;
            *p = nullptr;
            return LOUVAIN_OK;
        }
        if (need > g->arena_cap - g->arena_used)
            return fail(g, LOUVAIN_E_OOM,
                        "the allocation-free entry point's scratch (" + std::to_string(g->arena_cap) +
                            " bytes) cannot hold this run: " + std::to_string(g->arena_used + need) + " bytes needed");
        *p = (T *)(g->arena + g->arena_used);
        g->arena_used += need;
        return LOUVAIN_OK;
    }
    void *q = nullptr;
    if (pool().get(&q, bytes, g->dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(g, LOUVAIN_E_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    g->owned.push_back({q, bytes});
    *p = (T *)q;
    return LOUVAIN_OK;
}

void release_all(G *g)
{
    if (g->st) (void)hipStreamSynchronize(g->st);
    if (g->gst) (void)hipStreamSynchronize(g->gst);
    for (G::Stage *sg : {&g->stage_colored, &g->stage_batch})
        if (sg->exec) {
            (void)hipGraphExecDestroy(sg->exec);
            sg->exec = nullptr;
        }
    for (auto &ev : g->gev)
        if (ev) {
            (void)hipEventDestroy(ev);
            ev = nullptr;
        }
    if (g->gst) {
        (void)hipStreamDestroy(g->gst);
        g->gst = nullptr;
    }
    if (!g->arena)
        for (auto &b : g->owned) pool().put(b.first, b.second, g->dev);
    g->owned.clear();
    for (auto ev : g->event_pool) (void)hipEventDestroy(ev);
    for (auto &p : g->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    g->event_pool.clear();
    g->pending.clear();
}

louvain_status sync(G *g)
{
    HIPCHK(g, hipStreamSynchronize(g->st));
    HIPCHK(g, hipGetLastError());
    return LOUVAIN_OK;
}

// ---- profiling ----------------------------------------------------------------
const char *kNames[] = {"sweep_small_bins1to5", "sweep_large_bins6to7_hub_partition", "sweep_all_bins_small_group",
                        "sweep_hub_aggregate_decide", "commit", "coarsen", "color", "sweep_pack_communities",
                        "sweep_bin8"};
enum { PR_SMALL = 0, PR_LARGE = 1, PR_ALL = 2, PR_HUB_AGG = 3, PR_COMMIT = 4, PR_COARSEN = 5, PR_COLOR = 6,
       PR_PACK = 7, PR_BIN8 = 8, PR_COUNT = 9 };
constexpr double SMALL_GROUP = 65536; // vertices: one fused launch below this

hipEvent_t take_event(G *g)
{
    if (!g->event_pool.empty()) {
        hipEvent_t e = g->event_pool.back();
        g->event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    (void)hipEventCreate(&e);
    return e;
}

struct ProfScope {
    G *g;
    int rec;
    hipEvent_t a{}, b{};
    double bytes, entries;
    int slot;  // bit mask of the stats slots (bins) the launch covers, -1: none
    bool from_stats;
    ProfScope(G *g_, int rec_, double bytes_ = 0, double entries_ = 0, int slot_ = -1)
        : g(g_), rec(rec_), bytes(bytes_), entries(entries_), slot(slot_), from_stats(slot_ >= 0)
    {
        if (g->prof) {
            a = take_event(g);
            (void)hipEventRecord(a, g->st);
        }
    }
    ~ProfScope()
    {
        if (!g->prof) return;
        b = take_event(g);
        (void)hipEventRecord(b, g->st);
        g->pending.push_back({a, b, rec, bytes, entries, slot, from_stats, g->singleton});
    }
};

// after a stream sync: fold pending event pairs into the records; sweep
// launches take entries and pairs from their stats slot (slot -> bytes)
void prof_collect(G *g, const lv::SweepStats *host_stats, int wb)
{
    if (!g->prof) return;
    bool slot_done[lv::NBINS] = {false};
    for (auto &p : g->pending) {
        float ms = 0;
        (void)hipEventElapsedTime(&ms, p.a, p.b);
        ProfRec &r = g->recs[p.rec];
        r.launches += 1;
        r.ms += ms;
        if (p.from_stats && host_stats) {
            // per vertex: list entry 4, offsets 16, comm 4, k 8, a[A] 8, sizes 8, comm_next 4
            // per entry: column 4 + weight wb + comm of the neighbour 4 (not read by a sweep
            // from the singleton partition, where it is the neighbour itself); per distinct
            // community: a 8
            // (a slot sums all launches of its bin since the last read: counted once)
            // hub rows: the entries are gathered by the pass-1 blocks of the
            // large (or all-bins) launch, the distinct pairs read by pass 2
            r.bytes += 52.0 * p.bytes;
            const bool hub_pass2 = p.rec == PR_HUB_AGG;
            for (int b = 0; b < lv::NBINS; ++b) {
                if (!((p.stat_slot >> b) & 1) || slot_done[b]) continue;
                const lv::SweepStats &s = host_stats[b];
                const bool hub = b >= 9;
                // hub entries: gathered by pass 1, or from singletons (no pass 1)
                // scanned by the pass-2 launch itself
                const bool entries_here = !hub || (p.singleton ? hub_pass2 : !hub_pass2);
                if (entries_here) {
                    r.bytes += ((p.singleton ? 4.0 : 8.0) + wb) * (double)s.entries;
                    r.entries += (double)s.entries;
                }
                if (!hub || hub_pass2) r.bytes += 8.0 * (double)s.pairs;
                if (!hub || hub_pass2) slot_done[b] = true;
            }
        } else {
            r.bytes += p.bytes;
            r.entries += p.entries;
        }
        g->event_pool.push_back(p.a);
        g->event_pool.push_back(p.b);
    }
    g->pending.clear();
}

// ---- graph / state helpers ------------------------------------------------------
int wbytes(const lv::Csr &c) { return c.wk == lv::W_UNIT ? 0 : (c.wk == lv::W_I32 ? 4 : 8); }

louvain_status init_state(G *g)
{
    const int64_t n = g->cur.n;
    lv::iota_i32(g->comm_prev, n, g->st);
    lv::iota_i32(g->comm_next, n, g->st);
    lv::fill<int32_t>(g->size, 1, n, g->st);
    if (n) HIPCHK(g, hipMemcpyAsync(g->a, g->k, n * sizeof(int64_t), hipMemcpyDeviceToDevice, g->st));
    g->sigma_in = g->self;
    g->singleton = true;
    ++g->epoch;
    g->colored = false;
    g->num_colors = 0;
    g->bins_valid = false;
    return LOUVAIN_OK;
}

louvain_status reset_level0(G *g)
{
    g->cur.n = g->n0;
    g->cur.nnz = g->nnz0;
    g->cur.off = g->off0;
    g->cur.col = g->col0;
    g->cur.w = g->w0;
    g->cur.wk = g->w0 ? lv::W_I32 : lv::W_UNIT;
    g->cur_buf = -1;
    g->level = 0;
    g->kmax = g->kmax0;
    g->self = g->self0;
    if (g->n0) HIPCHK(g, hipMemcpyAsync(g->k, g->k0, g->n0 * sizeof(int64_t), hipMemcpyDeviceToDevice, g->st));
    lv::iota_i32(g->orig_map, g->n0, g->st);
    return init_state(g);
}

bool wide_gains(const G *g) { return (i128)g->two_m * (i128)g->kmax >= ((i128)1 << 62); }

void release_buffer(G *g, void *p)
{
    if (g->arena) return; // carved from the scratch: nothing to give back
    for (auto it = g->owned.begin(); it != g->owned.end(); ++it)
        if (it->first == p) {
            pool().put(it->first, it->second, g->dev);
            g->owned.erase(it);
            return;
        }
}

// sorts the current graph's vertices by (group, degree bin); group = colour or none
louvain_status tune_lanes(G *g);

// by_color: one group per colour class; mask_inactive (batched form): the
// vertices of graphs that stopped sweeping are left out of every bin
louvain_status build_bins(G *g, bool by_color, bool mask_inactive = false)
{
    const int64_t n = g->cur.n;
    const int groups = by_color ? g->num_colors : 1;
    const int64_t nkeys = 16 * (int64_t)groups;
    if (nkeys > g->bin_hist_cap) return fail(g, LOUVAIN_E_STATE, "bin key capacity exceeded");
    lv::bin_keys(g->cur, by_color ? g->color : nullptr, g->keys, g->vals, g->st, mask_inactive ? g->b_gid : nullptr,
                 mask_inactive ? g->b_active : nullptr);
    lv::radix_sort(g->keys, g->keys_alt, g->vals, g->vals_alt, n, 4 + (by_color ? bits_for(groups) : 0), g->scratch,
                   g->st);
    lv::narrow_ids(g->vals, g->bin_verts, n, g->st);
    lv::key_offsets(g->keys, n, nkeys, g->bin_offd, g->st);
    lv::hub_prefix(g->cur, g->bin_verts, n, g->cpre, g->bpre, g->xpre, g->scratch, g->st);
    g->bin_off.assign(nkeys + 1, 0);
    HIPCHK(g, hipMemcpyAsync(g->bin_off.data(), g->bin_offd, (nkeys + 1) * sizeof(int64_t), hipMemcpyDeviceToHost,
                             g->st));
    int64_t tot[3] = {0, 0, 0}; // chunks, buckets, bucket boundaries
    HIPCHK(g, hipMemcpyAsync(&tot[0], g->cpre + n, sizeof(int64_t), hipMemcpyDeviceToHost, g->st));
    HIPCHK(g, hipMemcpyAsync(&tot[1], g->bpre + n, sizeof(int64_t), hipMemcpyDeviceToHost, g->st));
    HIPCHK(g, hipMemcpyAsync(&tot[2], g->xpre + n, sizeof(int64_t), hipMemcpyDeviceToHost, g->st));
    louvain_status s = sync(g);
    if (s) return s;
    // hub position ranges (bins 9 and 10) per group
    std::vector<int64_t> idx;
    std::vector<int> with_hubs;
    for (int grp = 0; grp < groups; ++grp) {
        const int64_t hs = g->bin_off[grp * 16 + 9], he = g->bin_off[grp * 16 + 11];
        if (he > hs) {
            with_hubs.push_back(grp);
            idx.push_back(hs);
            idx.push_back(he);
        }
    }
    g->hub_groups.assign(groups, lv::HubArgs{});
    const int64_t pairs = tot[0] * lv::HUB_CHUNK;
    if (pairs > g->pcap) {
        release_buffer(g, g->pkey);
        release_buffer(g, g->pval);
        release_buffer(g, g->chunk_rec);
        const int64_t cap = pairs + pairs / 4 + lv::HUB_CHUNK;
        if ((s = alloc(g, &g->pkey, cap)) || (s = alloc(g, &g->pval, cap)) ||
            (s = alloc(g, &g->chunk_rec, cap / lv::HUB_CHUNK + 1)))
            return s;
        g->pcap = cap;
    }
    if (tot[2] > g->xcap) {
        release_buffer(g, g->boff);
        const int64_t cap = tot[2] + tot[2] / 4 + 1024;
        if ((s = alloc(g, &g->boff, cap))) return s;
        g->xcap = cap;
    }
    if (tot[1] > g->qcap) {
        release_buffer(g, g->hpart);
        release_buffer(g, g->hself);
        release_buffer(g, g->bucket_rec);
        const int64_t cap = tot[1] + tot[1] / 4 + 64;
        if ((s = alloc(g, &g->hpart, lv::HUB_REC * cap)) || (s = alloc(g, &g->hself, cap)) ||
            (s = alloc(g, &g->bucket_rec, cap)))
            return s;
        g->qcap = cap;
        lv::fill<int64_t>(g->hself, 0, cap, g->st); // the hub decisions leave it zero
    }
    if (!with_hubs.empty()) {
        lv::hub_owners(g->bin_verts, g->cur.off, g->cpre, g->bpre, g->xpre, n, g->chunk_rec, g->bucket_rec, g->st);
        const int64_t m = (int64_t)idx.size();
        // gather cpre and bpre at the range ends: device scratch in vals_alt (free here)
        int64_t *didx = g->vals_alt, *dout = g->vals_alt + m;
        HIPCHK(g, hipMemcpyAsync(didx, idx.data(), m * sizeof(int64_t), hipMemcpyHostToDevice, g->st));
        lv::gather_i64(g->cpre, didx, m, dout, g->st);
        lv::gather_i64(g->bpre, didx, m, dout + m, g->st);
        std::vector<int64_t> vals(2 * m);
        HIPCHK(g, hipMemcpyAsync(vals.data(), dout, 2 * m * sizeof(int64_t), hipMemcpyDeviceToHost, g->st));
        if ((s = sync(g))) return s;
        for (size_t t = 0; t < with_hubs.size(); ++t) {
            lv::HubArgs &h = g->hub_groups[with_hubs[t]];
            h.verts = g->bin_verts;
            h.s = idx[2 * t];
            h.e = idx[2 * t + 1];
            h.cpre = g->cpre;
            h.bpre = g->bpre;
            h.xpre = g->xpre;
            h.chunks = g->chunk_rec;
            h.buckets = g->bucket_rec;
            h.chunk0 = vals[2 * t];
            h.n_chunks = vals[2 * t + 1] - h.chunk0;
            h.bucket0 = vals[m + 2 * t];
            h.n_buckets = vals[m + 2 * t + 1] - h.bucket0;
            h.pkey = g->pkey;
            h.pval = g->pval;
            h.boff = g->boff;
            h.part = g->hpart;
            h.self = g->hself;
        }
    }
    g->bin_groups = groups;
    g->bins_colored = by_color;
    g->bins_valid = true;
    ++g->epoch;
    // lanes per vertex, chosen at the start of a phase (singleton state) from
    // the process-wide choices, timing the ones not made yet
    if (g->tune && g->singleton && !g->prof) return tune_lanes(g);
    return LOUVAIN_OK;
}

// Runs the launches of f() as one stage.  Outside profiling, and once the
// state is past the singleton partition, the first call of an epoch captures
// them (on the private stream) into a HIP graph; every call then launches the
// graph, ordered after the work already on the handle's stream and before
// the work that follows.  f() must only enqueue kernels.
template <class F> louvain_status run_stage(G *g, G::Stage &sg, F f)
{
    if (g->prof || !g->graphs_ok || g->singleton || (&sg == &g->stage_colored && !g->graph_colored)) {
        f();
        return LOUVAIN_OK;
    }
    if (!g->gst) {
        if (hipStreamCreateWithFlags(&g->gst, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&g->gev[0], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&g->gev[1], hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            g->graphs_ok = false;
            f();
            return LOUVAIN_OK;
        }
    }
    if (!sg.exec || sg.epoch != g->epoch) {
        if (sg.exec) {
            (void)hipGraphExecDestroy(sg.exec);
            sg.exec = nullptr;
        }
        hipStream_t main = g->st;
        hipGraph_t graph = nullptr;
        g->st = g->gst;
        hipError_t e = hipStreamBeginCapture(g->gst, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            f();
            e = hipStreamEndCapture(g->gst, &graph);
        }
        g->st = main;
        if (e == hipSuccess) e = hipGraphInstantiate(&sg.exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            sg.exec = nullptr;
            g->graphs_ok = false;
            f();
            return LOUVAIN_OK;
        }
        sg.epoch = g->epoch;
    }
    HIPCHK(g, hipEventRecord(g->gev[0], g->st));
    HIPCHK(g, hipStreamWaitEvent(g->gst, g->gev[0], 0));
    HIPCHK(g, hipGraphLaunch(sg.exec, g->gst));
    HIPCHK(g, hipEventRecord(g->gev[1], g->gst));
    HIPCHK(g, hipStreamWaitEvent(g->st, g->gev[1], 0));
    return LOUVAIN_OK;
}

// launches the sweep kernels of one group (all bins); per-bin stats slots
// the sweep arguments of the current state
lv::SweepArgs sweep_args(G *g, int singlet)
{
    lv::SweepArgs a;
    a.g = g->cur;
    a.comm_prev = g->comm_prev;
    a.comm_next = g->comm_next;
    a.a = g->a;
    a.size = g->size;
    a.k = g->k;
    a.two_m = g->two_m;
    a.singlet = singlet;
    a.singleton = g->singleton ? 1 : 0;
    a.gid = g->b_gid;
    a.two_m_g = g->b_two_m;
    a.active_g = g->b_active;
    a.gstats = g->b_gstats;
    a.stats = g->stats + 10 * lv::STAT_REP;
    return a;
}

// decide_hubs = false: the hub decisions are left to the commit of the group.
// plain: a synchronous sweep of every vertex (no colour classes), whose
// community totals stay fixed during the launches
void sweep_group(G *g, int group, int singlet, bool decide_hubs = true, bool plain = false)
{
    lv::SweepArgs a = sweep_args(g, singlet);
    const bool wide = wide_gains(g);
    const bool narrow = g->kmax <= (int64_t)UINT32_MAX; // hub sums e <= k_i fit 32 bits
    lv::FusedBins f;
    double cnt_small = 0, cnt_large = 0;
    for (int b = 1; b <= 8; ++b) {
        const int64_t s = g->bin_off[group * 16 + b], e = g->bin_off[group * 16 + b + 1];
        f.bins[b].verts = g->bin_verts + s;
        f.bins[b].count = e - s;
        f.bins[b].stats = g->stats + b * lv::STAT_REP;
        f.lanes[b] = g->lanes[b];
        (b <= 5 ? cnt_small : cnt_large) += (double)(e - s);
    }
    const lv::HubArgs &h = g->hub_groups[group];
    const double nhub = (double)(h.e > h.s ? h.e - h.s : 0);
    if (cnt_small + cnt_large + nhub <= SMALL_GROUP) {
        // small group (typical late colour class): one launch for every bin
        ProfScope ps(g, PR_ALL, cnt_small + cnt_large, 0, 0x7fe);
        lv::sweep_all(a, f, h, wide, narrow, g->st);
    } else {
        if (plain && !g->singleton && !g->b_gid && !wide && g->two_m <= (int64_t)UINT32_MAX) {
            // each vertex's community and that community's total, side by
            // side, so that the rows of bins 1..8 read both in one gather
            // (keys_alt is free between the binning and the rebuild)
            ProfScope ps(g, PR_PACK, 20.0 * (double)g->cur.n, 0);
            lv::pack_communities(g->comm_prev, g->a, g->cur.n, g->keys_alt, g->st);
            a.cpack = g->keys_alt;
        }
        {
            ProfScope ps(g, PR_SMALL, cnt_small, 0, 0x3e);
            lv::sweep_small(a, f, wide, g->st);
        }
        const double cnt8 = (double)f.bins[8].count;
        if (cnt8 > 0) {
            ProfScope ps(g, PR_BIN8, cnt8, 0, 0x100);
            lv::sweep_bin8(a, f, wide, narrow, g->st);
        }
        ProfScope ps(g, PR_LARGE, cnt_large - cnt8, 0, 0x6c0);
        lv::sweep_large(a, f, h, wide, narrow, g->st);
    }
    if (h.e > h.s) {
        ProfScope ps(g, PR_HUB_AGG, nhub, 0, 0x600);
        lv::sweep_hub_agg(a, h, wide, narrow, decide_hubs, g->st);
    }
}

// ---- autotuning of the lanes per vertex ---------------------------------------
// Process-wide choices by (device, weight kind, bin, log2 of the bin's
// vertices): the first handle that sees a bin of that kind and size times
// every choice of kLaneChoices on it and keeps the fastest.
struct LaneCache {
    std::mutex mu;
    std::map<std::tuple<int, int, int, int>, int> lanes;
};
LaneCache &lane_cache()
{
    static LaneCache *c = new LaneCache(); // lives until process end
    return *c;
}

int lg_bucket(int64_t x)
{
    int b = 0;
    while (((int64_t)1 << (b + 1)) <= x) ++b;
    return b;
}

// Chooses g->lanes for the bins of group 0.  A trial is one sweep launch of
// that bin alone: it writes comm_next of those vertices and statistics, and
// nothing else (no commit), so the state is unchanged; the statistics are
// cleared before every real sweep.
louvain_status tune_lanes(G *g)
{
    constexpr int64_t MIN_VERTICES = 16384; // smaller bins keep the default
    const lv::SweepArgs a = sweep_args(g, 1);
    const bool wide = wide_gains(g);
    const bool narrow = g->kmax <= (int64_t)UINT32_MAX;
    const lv::HubArgs none;
    for (int b = 1; b <= 6; ++b) {
        const int64_t s = g->bin_off[b], e = g->bin_off[b + 1];
        if (e - s < MIN_VERTICES || lv::kLaneChoices[b][1] == 0) continue;
        const auto key = std::make_tuple(g->dev, (int)g->cur.wk, b, lg_bucket(e - s));
        {
            std::lock_guard<std::mutex> lk(lane_cache().mu);
            auto it = lane_cache().lanes.find(key);
            if (it != lane_cache().lanes.end()) {
                g->lanes[b] = it->second;
                continue;
            }
        }
        int best = g->lanes[b];
        float best_ms = 1e30f;
        for (int c = 0; c < 4 && lv::kLaneChoices[b][c]; ++c) {
            lv::FusedBins f;
            f.bins[b].verts = g->bin_verts + s;
            f.bins[b].count = e - s;
            f.bins[b].stats = g->stats + b * lv::STAT_REP;
            f.lanes[b] = lv::kLaneChoices[b][c];
            float ms_min = 1e30f;
            for (int rep = 0; rep < 3; ++rep) { // the first is a warm-up
                hipEvent_t e0 = take_event(g), e1 = take_event(g);
                HIPCHK(g, hipEventRecord(e0, g->st));
                if (b <= 5) lv::sweep_small(a, f, wide, g->st);
                else lv::sweep_large(a, f, none, wide, narrow, g->st);
                HIPCHK(g, hipEventRecord(e1, g->st));
                HIPCHK(g, hipEventSynchronize(e1));
                float ms = 0;
                HIPCHK(g, hipEventElapsedTime(&ms, e0, e1));
                if (rep) ms_min = std::min(ms_min, ms);
                g->event_pool.push_back(e0);
                g->event_pool.push_back(e1);
            }
            if (std::getenv("LOUVAIN_TUNE_LOG"))
                std::fprintf(stderr, "louvain tune:   bin %d lanes %d: %.3f ms\n", b, lv::kLaneChoices[b][c], ms_min);
            if (ms_min < best_ms) {
                best_ms = ms_min;
                best = lv::kLaneChoices[b][c];
            }
        }
        g->lanes[b] = best;
        if (std::getenv("LOUVAIN_TUNE_LOG"))
            std::fprintf(stderr, "louvain tune: level %d bin %d (%lld vertices, weight kind %d): %d lanes, %.3f ms\n",
                         g->level, b, (long long)(e - s), (int)g->cur.wk, best, best_ms);
        std::lock_guard<std::mutex> lk(lane_cache().mu);
        lane_cache().lanes[key] = best;
    }
    lv::clear_stats(g->stats, lv::NBINS * lv::STAT_REP, g->st);
    return sync(g);
}

// sweep statistics summed over bins
struct SweepSum {
    int64_t moves = 0, sigma_prev = 0, dsigma = 0, pairs = 0, entries = 0;
};

louvain_status read_stats(G *g, SweepSum &out, lv::SweepStats *host)
{
    std::vector<lv::SweepStats> rep(lv::NBINS * lv::STAT_REP);
    HIPCHK(g, hipMemcpyAsync(rep.data(), g->stats, rep.size() * sizeof(lv::SweepStats), hipMemcpyDeviceToHost,
                             g->st));
    louvain_status s = sync(g);
    if (s) return s;
    for (int b = 0; b < lv::NBINS; ++b) {
        host[b] = lv::SweepStats{};
        for (int r = 0; r < lv::STAT_REP; ++r) {
            const lv::SweepStats &x = rep[b * lv::STAT_REP + r];
            host[b].moves += x.moves;
            host[b].sigma_prev += x.sigma_prev;
            host[b].dsigma += x.dsigma;
            host[b].pairs += x.pairs;
            host[b].entries += x.entries;
        }
    }
    out = SweepSum();
    for (int b = 0; b < lv::NBINS; ++b) {
        out.moves += host[b].moves;
        out.sigma_prev += host[b].sigma_prev;
        out.dsigma += host[b].dsigma;
        out.pairs += host[b].pairs;
        out.entries += host[b].entries;
    }
    return LOUVAIN_OK;
}

louvain_status read_i128(G *g, const int64_t *dptr, i128 &v)
{
    int64_t h[2];
    HIPCHK(g, hipMemcpyAsync(h, dptr, sizeof(h), hipMemcpyDeviceToHost, g->st));
    louvain_status s = sync(g);
    if (s) return s;
    v = (i128)(((u128)(uint64_t)h[1] << 64) | (u128)(uint64_t)h[0]);
    return LOUVAIN_OK;
}

louvain_status sum_sq(G *g, const int64_t *x, int64_t n, i128 &out)
{
    lv::sum_squares(x, n, g->dscal + 4, g->scratch, g->st);
    return read_i128(g, g->dscal + 4, out);
}

// commit of an uncoloured sweep: the vertices of bins 1..10 (bin 0 holds the
// rows without entries, which have no candidate and never move)
louvain_status commit_all(G *g)
{
    const int64_t s = g->bin_off[1], e = g->bin_off[11];
    ProfScope ps(g, PR_COMMIT, 8.0 * (double)(e - s), 0);
    lv::commit(g->bin_verts + s, e - s, g->comm_prev, g->comm_next, g->k, g->a, g->size, g->st);
    g->singleton = false;
    return LOUVAIN_OK;
}

// keeps the current partition so that the next iteration can be undone
louvain_status save_partition(G *g)
{
    if (g->cur.n)
        HIPCHK(g, hipMemcpyAsync(g->comm_save, g->comm_prev, g->cur.n * sizeof(int32_t), hipMemcpyDeviceToDevice,
                                 g->st));
    return LOUVAIN_OK;
}

// an iteration that lost modularity is undone: every vertex goes back to its
// saved community, with the community degrees and sizes moved back alike
louvain_status undo_iteration(G *g)
{
    ProfScope ps(g, PR_COMMIT, 12.0 * (double)g->cur.n, 0);
    lv::commit(nullptr, g->cur.n, g->comm_prev, g->comm_save, g->k, g->a, g->size, g->st);
    return LOUVAIN_OK;
}

// colored iteration: classes in ascending colour, each synchronous on the
// state after the classes before it (Sec. 5.4 step 3)
louvain_status colored_iteration(G *g, int singlet, SweepSum &sum, lv::SweepStats *host)
{
    louvain_status st = run_stage(g, g->stage_colored, [&]() {
        lv::clear_stats(g->stats, lv::NBINS * lv::STAT_REP, g->st);
        const lv::SweepArgs a = sweep_args(g, singlet);
        const bool wide = wide_gains(g);
        for (int c = 0; c < g->num_colors; ++c) {
            sweep_group(g, c, singlet, false);
            const int64_t s = g->bin_off[c * 16], e = g->bin_off[c * 16 + 16];
            ProfScope ps(g, PR_COMMIT, 8.0 * (double)(e - s), 0);
            lv::commit_hubs(a, g->hub_groups[c], g->bin_verts + s, s, e - s, wide, g->st);
            g->singleton = false;
        }
    });
    if (st) return st;
    st = read_stats(g, sum, host);
    prof_collect(g, host, wbytes(g->cur));
    return st;
}

// whether the rebuild sums its pairs per tile before sorting.  The last
// sweep's count of distinct (vertex, community) pairs bounds the keys a
// tile can fold; measured on R-MAT 24, the sums pay below 90 % of the
// entries for weighted graphs (pairs at 66 %: 44 against 51 ms) and are even
// at 94 %, while unit weights sort their keys alone (no values), which wins
// near 100 % (44 against 74 ms); taken at 50 % there.  Always for the
// batched form.
bool tile_sums(const G *g)
{
    if (g->tile_sums_mode >= 0) return g->tile_sums_mode == 1;
    if (g->b_gid) return true;
    if (g->iters.empty()) return false;
    const int64_t pairs = g->iters.back().pairs, nnz = g->cur.nnz;
    return g->cur.wk == lv::W_UNIT ? 2 * pairs <= nnz : 10 * pairs <= 9 * nnz;
}

// rebuild the community graph of the current partition (Sec. 5.4 step 4)
// vf: comm is a vertex-following map (the rebuild compacts rows, no sort)
louvain_status coarsen_current(G *g, const int32_t *comm, int64_t &n_new, bool vf = false)
{
    const int dst = g->cur_buf == 0 ? 1 : 0;
    lv::CoarsenBufs b{g->flag, g->new_id, g->keys, g->keys_alt, g->vals, g->vals_alt, g->run, g->keys_words};
    int64_t nnz_new = 0;
    {
        ProfScope ps(g, PR_COARSEN, 0, (double)g->cur.nnz);
        const hipError_t e =
            vf ? lv::coarsen_vf(g->cur, comm, g->k, g->orig_map, g->n0, b, g->off_b[dst], g->col_b[dst], g->w_b[dst],
                                g->k, g->dscal, &n_new, &nnz_new, g->scratch, g->st)
               : lv::coarsen(g->cur, comm, g->orig_map, g->n0, b, g->off_b[dst], g->col_b[dst], g->w_b[dst], g->k,
                             g->dscal, &n_new, &nnz_new, g->scratch, g->st, tile_sums(g));
        if (e != hipSuccess) return hip_fail(g, e, "graph rebuild");
    }
    g->cur.n = n_new;
    g->cur.nnz = nnz_new;
    g->cur.off = g->off_b[dst];
    g->cur.col = g->col_b[dst];
    g->cur.w = g->w_b[dst];
    g->cur.wk = lv::W_I64;
    g->cur_buf = dst;
    g->level += 1;
    int64_t h[3];
    HIPCHK(g, hipMemcpyAsync(h, g->dscal, sizeof(h), hipMemcpyDeviceToHost, g->st));
    louvain_status s = sync(g);
    if (s) return s;
    prof_collect(g, nullptr, 0);
    if (h[0] != g->two_m) return fail(g, LOUVAIN_E_STATE, "internal error: 2m changed by coarsening");
    g->kmax = h[1];
    g->self = h[2];
    return init_state(g);
}

// vertex following before the first phase (Sec. 5.3): mode 1 single-degree
// vertices, one round; mode 2 chain compression, rounds until no vertex
// follows another.  after(n_before, n_after) runs after every rebuild (the
// batched form's bookkeeping).  *rounds_out: the rounds that rebuilt.
template <class F> louvain_status vertex_following(G *g, int mode, F after, int64_t *rounds_out)
{
    louvain_status s;
    int64_t rounds = 0;
    for (;;) {
        const int64_t n0 = g->cur.n;
        if (mode == 1) {
            lv::vf_map(g->cur, g->comm_prev, g->st);
        } else {
            lv::vf_chain_map(g->cur, g->k, g->two_m, g->b_gid, g->b_two_m, g->comm_prev, g->dscal + 12, g->scratch,
                             g->st);
            int64_t moved = 0;
            HIPCHK(g, hipMemcpyAsync(&moved, g->dscal + 12, sizeof(int64_t), hipMemcpyDeviceToHost, g->st));
            if ((s = sync(g))) return s;
            if (moved == 0) break;
        }
        int64_t nv = 0;
        if ((s = coarsen_current(g, g->comm_prev, nv, true))) return s;
        if ((s = after(n0, nv))) return s;
        ++rounds;
        if (mode == 1) break;
    }
    if (rounds_out) *rounds_out = rounds;
    return LOUVAIN_OK;
}

louvain_status do_color(G *g, uint64_t seed)
{
    {
        ProfScope ps(g, PR_COLOR, 0, (double)g->cur.nnz);
        const int64_t n = g->cur.n;
        const int64_t pairs = lv::color_chunk_pairs(g->cur), words = lv::color_bitmap_words(g->cur);
        louvain_status s;
        if (pairs > g->jp_chunk_cap) {
            release_buffer(g, g->jp_chunk);
            if ((s = alloc(g, &g->jp_chunk, 8 * pairs))) return s;
            g->jp_chunk_cap = pairs;
        }
        if (words > g->jp_bm_cap) {
            release_buffer(g, g->jp_bm);
            if ((s = alloc(g, &g->jp_bm, words))) return s;
            g->jp_bm_cap = words;
        }
        lv::ColorBufs c;
        c.color = g->color;
        c.cnt = g->jp_cnt;
        c.long_id = g->jp_cnt + n;
        c.light[0] = g->jp_light;
        c.light[1] = g->jp_light + 2 * n;
        c.counters = g->counters;
        c.chunk[0] = g->jp_chunk;
        c.chunk[1] = g->jp_chunk + 4 * g->jp_chunk_cap;
        c.bm = (unsigned long long *)g->jp_bm;
        g->num_colors = lv::color_jp(g->cur, seed, c, g->scratch, g->st);
        if (g->num_colors < 0) return hip_fail(g, hipGetLastError(), "coloring (copy or wait on the stream)");
    }
    louvain_status s = sync(g);
    if (s) return s;
    prof_collect(g, nullptr, 0);
    if ((int64_t)16 * g->num_colors > g->bin_hist_cap) {
        release_buffer(g, g->bin_hist);
        release_buffer(g, g->bin_offd);
        g->bin_hist_cap = (int64_t)16 * g->num_colors + 16;
        if ((s = alloc(g, &g->bin_hist, g->bin_hist_cap))) return s;
        if ((s = alloc(g, &g->bin_offd, g->bin_hist_cap + 1))) return s;
    }
    g->colored = true;
    g->bins_valid = false;
    return LOUVAIN_OK;
}

// balanced colouring of the current colouring (after do_color); *moved_out:
// the vertices that changed class
louvain_status do_balance(G *g, uint64_t seed, int64_t *moved_out)
{
    if (!g->colored) return fail(g, LOUVAIN_E_STATE, "balancing needs a colouring of the current graph");
    const int64_t n = g->cur.n;
    lv::BalanceBufs b;
    b.color = g->color;
    b.list = g->bin_verts;
    b.waiting = g->jp_cnt;
    b.prop = g->jp_cnt + n;
    b.taken = g->jp_cnt + 2 * n;
    b.before = g->jp_cnt + 3 * n;
    b.size = (int32_t *)g->jp_light; // ncolors <= n
    b.closed = g->bal_closed;
    b.keys = g->keys;
    b.keys_alt = g->keys_alt;
    b.vals = g->vals;
    b.vals_alt = g->vals_alt;
    b.first = g->bin_offd;
    int64_t moved;
    {
        ProfScope ps(g, PR_COLOR, 0, (double)g->cur.nnz);
        moved = lv::color_balance(g->cur, seed, g->num_colors, b, g->scratch, g->st);
    }
    if (moved == -2) return fail(g, LOUVAIN_E_INVALID_ARG, "balanced colouring takes at most 4096 colours");
    if (moved < 0) return hip_fail(g, hipGetLastError(), "balanced colouring (copy or wait on the stream)");
    prof_collect(g, nullptr, 0);
    g->bins_valid = false;
    if (moved_out) *moved_out = moved;
    return LOUVAIN_OK;
}

louvain_status check_handle(G *g)
{
    if (!g) return LOUVAIN_E_INVALID_ARG;
    if (g->poisoned) return fail(g, LOUVAIN_E_HIP, "handle unusable after an earlier HIP error");
    HIPCHK(g, hipSetDevice(g->dev));
    return LOUVAIN_OK;
}

louvain_status check_params(G *g, const louvain_params *p)
{
    if (!p) return fail(g, LOUVAIN_E_INVALID_ARG, "params is NULL");
    if (p->theta_color.den <= 0 || p->theta_final.den <= 0 || p->theta_color.num < 0 || p->theta_final.num < 0)
        return fail(g, LOUVAIN_E_INVALID_ARG, "thresholds need num >= 0 and den > 0");
    if (p->max_iter < 1 || p->max_phases < 1) return fail(g, LOUVAIN_E_INVALID_ARG, "max_iter and max_phases must be >= 1");
    if (p->vf < 0 || p->vf > 2) return fail(g, LOUVAIN_E_INVALID_ARG, "vf is 0, 1 or 2");
    if (p->threshold_mode != 0 && p->threshold_mode != 1) return fail(g, LOUVAIN_E_INVALID_ARG, "threshold_mode is 0 or 1");
    if (p->color_balance != 0 && p->color_balance != 1) return fail(g, LOUVAIN_E_INVALID_ARG, "color_balance is 0 or 1");
    return LOUVAIN_OK;
}

louvain_status copy_out(G *g, void *dst, const void *src, size_t bytes, uint32_t on_device)
{
    if (!dst || !bytes) return LOUVAIN_OK;
    HIPCHK(g, hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, g->st));
    return sync(g);
}

// ---- one uncolored phase with the look-ahead modularity --------------------------
// Sweep s reads C_{s-1}, so its gather also yields the internal weight of
// C_{s-1} and hence Q_{s-1}; the stop test for iteration s-1 is therefore
// taken after sweep s, whose moves are discarded if iteration s-1 was the last.
// If iteration s-1 lost modularity (against Q_{s-2}; Q_0 is the phase's
// start), it is undone from the partition saved before its commit, and the
// phase ends (Sec. 5.1: a phase continues only on a net gain).
louvain_status run_phase_plain(G *g, const louvain_params *p, louvain_ratio th, louvain_phase_stats &ph, i128 N0)
{
    lv::SweepStats host[lv::NBINS];
    std::vector<i128> S2;     // S2[t] = sum a^2 after iteration t
    std::vector<i128> N;      // N[t]
    std::vector<int64_t> mv;  // moves[t]
    i128 s2_0;
    louvain_status s = sum_sq(g, g->k, g->cur.n, s2_0);
    if (s) return s;
    S2.push_back(s2_0);
    N.push_back(N0);
    mv.push_back(0);
    const i128 D = (i128)g->two_m * g->two_m;
    int t_end = 0;
    for (int s_idx = 1;; ++s_idx) {
        lv::clear_stats(g->stats, lv::NBINS * lv::STAT_REP, g->st);
        sweep_group(g, 0, p->singlet_rule, true, true);
        SweepSum sum;
        if ((s = read_stats(g, sum, host))) return s;
        prof_collect(g, host, wbytes(g->cur));
        g->swept_entries += sum.entries;
        louvain_iter_stats rec{};
        if (s_idx >= 2) {
            N[s_idx - 1] = (i128)g->two_m * sum.sigma_prev - S2[s_idx - 1];
            g->iters.back().q_num = to_abi(N[s_idx - 1]);
            if (N[s_idx - 1] < N[s_idx - 2]) {
                g->lookahead_entries += sum.entries;
                if ((s = undo_iteration(g))) return s;
                ph.loss_undone = 1;
                t_end = s_idx - 1;
                break;
            }
            if (s_idx - 1 >= 2 && below_threshold(N[s_idx - 1], N[s_idx - 2], D, th, p->threshold_mode)) {
                g->lookahead_entries += sum.entries;
                t_end = s_idx - 1;
                break;
            }
            if (s_idx - 1 >= p->max_iter) { // only reached when the cap needed N of the last iteration
                g->lookahead_entries += sum.entries;
                ph.hit_max_iter = 1;
                t_end = s_idx - 1;
                break;
            }
        }
        mv.push_back(sum.moves);
        N.push_back(0);
        S2.push_back(0);
        rec.moves = sum.moves;
        rec.pairs = sum.pairs;
        rec.entries = sum.entries;
        g->iters.push_back(rec);
        if (sum.moves == 0) {
            N[s_idx] = N[s_idx - 1];
            S2[s_idx] = S2[s_idx - 1];
            g->iters.back().q_num = to_abi(N[s_idx]);
            t_end = s_idx;
            break;
        }
        if ((s = save_partition(g))) return s;
        commit_all(g);
        lv::sum_squares(g->a, g->cur.n, g->dscal + 4, g->scratch, g->st);
        if ((s = read_i128(g, g->dscal + 4, S2[s_idx]))) return s;
        prof_collect(g, nullptr, 0);
        // at the iteration cap, one more sweep (whose moves are discarded) yields N[s_idx]
    }
    ph.iterations = t_end;
    ph.q_num = to_abi(ph.loss_undone ? N[t_end - 1] : N[t_end]);
    // drop the look-ahead record if it was pushed
    while ((int64_t)g->iters.size() > ph.first_iter + t_end) g->iters.pop_back();
    // comm_next may hold a discarded look-ahead; resync it with comm_prev
    if (g->cur.n)
        HIPCHK(g, hipMemcpyAsync(g->comm_next, g->comm_prev, g->cur.n * sizeof(int32_t), hipMemcpyDeviceToDevice,
                                 g->st));
    return LOUVAIN_OK;
}

louvain_status run_phase_colored(G *g, const louvain_params *p, louvain_ratio th, louvain_phase_stats &ph, i128 N0)
{
    lv::SweepStats host[lv::NBINS];
    const i128 D = (i128)g->two_m * g->two_m;
    i128 N_prev = N0, N_t = N0;
    int64_t sigma = g->self;
    louvain_status s;
    int t = 0;
    for (;;) {
        ++t;
        SweepSum sum;
        if ((s = save_partition(g))) return s;
        if ((s = colored_iteration(g, p->singlet_rule, sum, host))) return s;
        g->swept_entries += sum.entries;
        i128 S2;
        if ((s = sum_sq(g, g->a, g->cur.n, S2))) return s;
        sigma += sum.dsigma;
        N_t = (i128)g->two_m * sigma - S2;
        louvain_iter_stats rec{};
        rec.moves = sum.moves;
        rec.q_num = to_abi(N_t);
        rec.pairs = sum.pairs;
        rec.entries = sum.entries;
        g->iters.push_back(rec);
        if (sum.moves == 0) break;
        if (N_t < N_prev) { // a loss (Sec. 5.1): back to the partition before this iteration
            if ((s = undo_iteration(g))) return s;
            ph.loss_undone = 1;
            N_t = N_prev;
            break;
        }
        if (t >= 2 && below_threshold(N_t, N_prev, D, th, p->threshold_mode)) break;
        if (t >= p->max_iter) {
            ph.hit_max_iter = 1;
            break;
        }
        N_prev = N_t;
    }
    ph.iterations = t;
    ph.q_num = to_abi(N_t);
    return LOUVAIN_OK;
}

} // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void louvain_params_default(louvain_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->vf = 0;
    p->color = 0;
    p->singlet_rule = 1;
    p->threshold_mode = 0;
    p->color_first_phase_only = 0;
    p->max_iter = 1000;
    p->max_phases = 100;
    p->theta_color = {1, 100};
    p->theta_final = {1, 1000000};
    p->color_cutoff = 100000;
    p->color_seed = 0x4C4F5556ull;
}

const char *louvain_last_error(louvain_graph_t g) { return g ? g->err.c_str() : g_init_error.c_str(); }

} // extern "C"

namespace {

// device buffers of a handle for a graph of n vertices and nnz entries
louvain_status alloc_buffers(G *g, int64_t n, int64_t nnz, bool weighted)
{
    louvain_status s;
    const int64_t big = (nnz > n ? nnz : n) + 1;
    g->keys_words = big;
    if ((s = alloc(g, &g->off0, n + 1)) || (s = alloc(g, &g->col0, nnz)) || (s = alloc(g, &g->k0, n)) ||
        (weighted && (s = alloc(g, &g->w0, nnz))))
        return s;
    for (int b = 0; b < 2; ++b)
        if ((s = alloc(g, &g->off_b[b], n + 1)) || (s = alloc(g, &g->col_b[b], nnz)) ||
            (s = alloc(g, &g->w_b[b], nnz)))
            return s;
    if ((s = alloc(g, &g->k, n)) || (s = alloc(g, &g->a, n)) || (s = alloc(g, &g->comm_prev, n)) ||
        (s = alloc(g, &g->comm_next, n)) || (s = alloc(g, &g->comm_save, n)) || (s = alloc(g, &g->size, n)) ||
        (s = alloc(g, &g->orig_map, n)) ||
        (s = alloc(g, &g->color, n)) || (s = alloc(g, &g->jp_cnt, 5 * n)) || (s = alloc(g, &g->jp_light, 4 * n)) || (s = alloc(g, &g->counters, 16)) || (s = alloc(g, &g->keys, big)) ||
        (s = alloc(g, &g->keys_alt, big)) || (s = alloc(g, &g->vals, big)) || (s = alloc(g, &g->vals_alt, big)) ||
        (s = alloc(g, &g->run, big)) || (s = alloc(g, &g->bin_verts, n)) || (s = alloc(g, &g->cpre, n + 1)) ||
        (s = alloc(g, &g->bpre, n + 1)) || (s = alloc(g, &g->xpre, n + 1)) || (s = alloc(g, &g->flag, n + 1)) ||
        (s = alloc(g, &g->new_id, n + 1)) || (s = alloc(g, &g->stats, lv::NBINS * lv::STAT_REP)) ||
        (s = alloc(g, &g->dscal, 16)) || (s = alloc(g, &g->vflag, 4)) || (s = alloc(g, &g->bal_closed, 64)))
        return s;
    g->bin_hist_cap = 16 * 64;
    if ((s = alloc(g, &g->bin_hist, g->bin_hist_cap)) || (s = alloc(g, &g->bin_offd, g->bin_hist_cap + 1)))
        return s;
    const int64_t part = lv::radix_partials_needed(big) + lv::scan_partials_needed(256 * (big / 4096 + 1)) +
                         lv::scan_partials_needed(big) + 4096;
    if ((s = alloc(g, &g->scratch.part, part))) return s;
    g->scratch.part_cap = part;
    if ((s = alloc(g, &g->scratch.scalar, 8))) return s;
    if ((s = alloc(g, &g->scratch.rep, 8 * lv::RED_REP + 8))) return s;
    return LOUVAIN_OK;
}

// environment choices of a new handle
void read_env(G *g)
{
    // LOUVAIN_HIP_GRAPHS: 0 no graph capture, 1 (default) the batched
    // sweep stage, 2 also the colour classes of an iteration
    const char *env = std::getenv("LOUVAIN_HIP_GRAPHS");
    const int mode = env && env[0] >= '0' && env[0] <= '2' ? env[0] - '0' : 1;
    g->graphs_ok = mode > 0;
    g->graph_colored = mode > 1;
    const char *tune = std::getenv("LOUVAIN_AUTOTUNE");
    g->tune = !(tune && tune[0] == '0');
    // LOUVAIN_LANES=l1,l2,...: fixed lanes per vertex for bins 1, 2, ...
    // (each one of the bin's choices; no tuning)
    if (const char *ln = std::getenv("LOUVAIN_LANES")) {
        int b = 1;
        for (const char *q = ln; *q && b <= 8; ++b) {
            const int v = std::atoi(q);
            for (int c = 0; c < 4 && lv::kLaneChoices[b][c]; ++c)
                if (lv::kLaneChoices[b][c] == v) g->lanes[b] = v;
            while (*q && *q != ',') ++q;
            if (*q == ',') ++q;
        }
        g->tune = false;
    }
    // LOUVAIN_TILE_SUMS: 0 never sum the rebuild's pairs per tile, 1 always;
    // unset: by the last sweep's pair count
    const char *ts = std::getenv("LOUVAIN_TILE_SUMS");
    g->tile_sums_mode = (ts && (ts[0] == '0' || ts[0] == '1')) ? ts[0] - '0' : -1;
}

// copies (or validates in place) the input CSR into the handle's buffers,
// computes degrees and 2m and sets the first phase's singleton state
louvain_status ingest(G *g, int64_t n, int64_t nnz, const int64_t *offsets, const int32_t *cols,
                      const int32_t *weights, uint32_t flags)
{
    const bool dev_ptrs = flags & LOUVAIN_DEVICE_PTRS;
    g->n0 = n;
    g->nnz0 = nnz;
    g->recs.resize(PR_COUNT);
    for (int r = 0; r < PR_COUNT; ++r) g->recs[r].name = kNames[r];

    const hipMemcpyKind kind = dev_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (hipMemcpyAsync(g->off0, offsets, (n + 1) * sizeof(int64_t), kind, g->st) != hipSuccess ||
        (nnz && hipMemcpyAsync(g->col0, cols, nnz * sizeof(int32_t), kind, g->st) != hipSuccess) ||
        (weights && nnz && hipMemcpyAsync(g->w0, weights, nnz * sizeof(int32_t), kind, g->st) != hipSuccess)) {
        (void)hipGetLastError();
        g->err = "copy of the input CSR failed";
        return LOUVAIN_E_HIP;
    }
    lv::Csr in;
    in.n = n;
    in.nnz = nnz;
    in.off = g->off0;
    in.col = g->col0;
    in.w = g->w0;
    in.wk = g->w0 ? lv::W_I32 : lv::W_UNIT;
    static const char *why[] = {"", "offsets not monotone or not spanning [0, nnz]", "column out of range",
                                "columns not strictly ascending within a row", "weight below 1",
                                "graph not symmetric (missing mirror entry or different weight)"};
    const bool full = (flags & LOUVAIN_VALIDATE) != 0;
    {
        // offsets always, then with LOUVAIN_VALIDATE order, weights and
        // symmetry; without it the column range is checked by the degree pass
        // (which indexes nothing with a column), before any kernel that does
        int32_t code = 0;
        lv::validate_csr(in, g->vflag, g->st);
        if (hipMemcpyAsync(&code, g->vflag, sizeof(code), hipMemcpyDeviceToHost, g->st) != hipSuccess ||
            hipStreamSynchronize(g->st) != hipSuccess) {
            g->err = "validation failed to run";
            return LOUVAIN_E_HIP;
        }
        if (code == 0 && full) {
            lv::validate_entries(in, true, g->vflag, g->st);
            if (hipMemcpyAsync(&code, g->vflag, sizeof(code), hipMemcpyDeviceToHost, g->st) != hipSuccess ||
                hipStreamSynchronize(g->st) != hipSuccess) {
                g->err = "validation failed to run";
                return LOUVAIN_E_HIP;
            }
        }
        if (code != 0) {
            g->err = std::string("invalid CSR: ") + why[code > 0 && code < 6 ? code : 0];
            return LOUVAIN_E_BAD_CSR;
        }
    }
    lv::degrees(in, g->k0, g->dscal, g->scratch, g->st, full ? nullptr : g->vflag);
    int64_t h[3];
    int32_t range_code = 0;
    if (hipMemcpyAsync(h, g->dscal, sizeof(h), hipMemcpyDeviceToHost, g->st) != hipSuccess ||
        hipMemcpyAsync(&range_code, g->vflag, sizeof(range_code), hipMemcpyDeviceToHost, g->st) != hipSuccess ||
        hipStreamSynchronize(g->st) != hipSuccess) {
        g->err = "degree computation failed";
        return LOUVAIN_E_HIP;
    }
    if (range_code != 0) {
        g->err = std::string("invalid CSR: ") + why[range_code > 0 && range_code < 6 ? range_code : 0];
        return LOUVAIN_E_BAD_CSR;
    }
    g->two_m = h[0];
    g->kmax0 = h[1];
    g->self0 = h[2];
    if (g->two_m < 0 || g->two_m >= ((int64_t)1 << 62)) {
        g->err = "2m >= 2^62";
        return LOUVAIN_E_OVERFLOW;
    }
    louvain_status s;
    if ((s = reset_level0(g)) || (s = sync(g))) return s;
    return LOUVAIN_OK;
}

// argument checks shared by the ingest entry points
louvain_status check_csr_args(int64_t n, int64_t nnz, const int64_t *offsets, const int32_t *cols, uint32_t flags)
{
    if (n < 0 || nnz < 0) return fail(nullptr, LOUVAIN_E_INVALID_ARG, "negative size");
    if (n >= ((int64_t)1 << 31) - 1) return fail(nullptr, LOUVAIN_E_INVALID_ARG, "n must be below 2^31 - 1");
    if (!offsets) return fail(nullptr, LOUVAIN_E_INVALID_ARG, "offsets is NULL");
    if (nnz > 0 && !cols) return fail(nullptr, LOUVAIN_E_INVALID_ARG, "cols is NULL");
    if (flags & ~(LOUVAIN_DEVICE_PTRS | LOUVAIN_VALIDATE)) return fail(nullptr, LOUVAIN_E_INVALID_ARG, "unknown flags");
    if (!(flags & LOUVAIN_DEVICE_PTRS)) {
        if (offsets[0] != 0 || offsets[n] != nnz)
            return fail(nullptr, LOUVAIN_E_BAD_CSR, "offsets[0] must be 0 and offsets[n] must equal nnz");
    }
    return LOUVAIN_OK;
}

} // namespace

extern "C" {

louvain_status louvain_init_csr(int64_t n, int64_t nnz, const int64_t *offsets, const int32_t *cols,
                                const int32_t *weights, uint32_t flags, void *hip_stream, louvain_graph_t *out)
{
    g_init_error.clear();
    if (!out) return fail(nullptr, LOUVAIN_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    louvain_status s = check_csr_args(n, nnz, offsets, cols, flags);
    if (s) return s;
    G *g = new G();
    g->st = (hipStream_t)hip_stream;
    if (const hipError_t e = hipGetDevice(&g->dev)) {
        delete g;
        return fail(nullptr, LOUVAIN_E_HIP, std::string("hipGetDevice failed: ") + hipGetErrorString(e));
    }
    auto bail = [&](louvain_status st) {
        g_init_error = g->err;
        release_all(g);
        delete g;
        return st;
    };
    if ((s = alloc_buffers(g, n, nnz, weights != nullptr))) return bail(s);
    read_env(g);
    if ((s = ingest(g, n, nnz, offsets, cols, weights, flags))) return bail(s);
    *out = g;
    return LOUVAIN_OK;
}

void louvain_destroy(louvain_graph_t g)
{
    if (!g) return;
    (void)hipSetDevice(g->dev);
    release_all(g);
    delete g;
}

louvain_status louvain_vf(louvain_graph_t g, int64_t *n_new_out)
{
    louvain_status s = check_handle(g);
    if (s) return s;
    if (g->level != 0) return fail(g, LOUVAIN_E_STATE, "vertex following applies to the input graph only");
    if ((s = vertex_following(g, 1, [](int64_t, int64_t) { return LOUVAIN_OK; }, nullptr))) return s;
    if (n_new_out) *n_new_out = g->cur.n;
    return LOUVAIN_OK;
}

louvain_status louvain_vf_chain(louvain_graph_t g, int64_t *n_new_out, int64_t *rounds_out)
{
    louvain_status s = check_handle(g);
    if (s) return s;
    if (g->level != 0) return fail(g, LOUVAIN_E_STATE, "vertex following applies to the input graph only");
    if ((s = vertex_following(g, 2, [](int64_t, int64_t) { return LOUVAIN_OK; }, rounds_out))) return s;
    if (n_new_out) *n_new_out = g->cur.n;
    return LOUVAIN_OK;
}

louvain_status louvain_color(louvain_graph_t g, uint64_t seed, int32_t *num_colors_out)
{
    louvain_status s = check_handle(g);
    if (s) return s;
    if ((s = do_color(g, seed))) return s;
    if (num_colors_out) *num_colors_out = g->num_colors;
    return LOUVAIN_OK;
}

louvain_status louvain_color_balance(louvain_graph_t g, uint64_t seed, int64_t *moved_out)
{
    louvain_status s = check_handle(g);
    if (s) return s;
    return do_balance(g, seed, moved_out);
}

louvain_status louvain_sweep(louvain_graph_t g, const louvain_params *p, louvain_iter_stats *out)
{
    louvain_status s = check_handle(g);
    if (s) return s;
    if (!p) return fail(g, LOUVAIN_E_INVALID_ARG, "params is NULL");
    const bool colored = p->color && g->colored;
    if (!g->bins_valid || g->bins_colored != colored)
        if ((s = build_bins(g, colored))) return s;
    lv::SweepStats host[lv::NBINS];
    SweepSum sum;
    if (colored) {
        if ((s = colored_iteration(g, p->singlet_rule, sum, host))) return s;
    } else {
        lv::clear_stats(g->stats, lv::NBINS * lv::STAT_REP, g->st);
        sweep_group(g, 0, p->singlet_rule, true, true);
        if ((s = read_stats(g, sum, host))) return s;
        prof_collect(g, host, wbytes(g->cur));
        commit_all(g);
    }
    i128 S2;
    if ((s = sum_sq(g, g->a, g->cur.n, S2))) return s;
    lv::internal_weight(g->cur, g->comm_prev, g->dscal + 8, g->scratch, g->st);
    int64_t sigma = 0;
    HIPCHK(g, hipMemcpyAsync(&sigma, g->dscal + 8, sizeof(int64_t), hipMemcpyDeviceToHost, g->st));
    if ((s = sync(g))) return s;
    prof_collect(g, nullptr, 0);
    g->sigma_in = sigma;
    if (out) {
        std::memset(out, 0, sizeof(*out));
        out->moves = sum.moves;
        out->pairs = sum.pairs;
        out->entries = sum.entries;
        out->q_num = to_abi(g->two_m ? (i128)g->two_m * sigma - S2 : (i128)0);
    }
    return LOUVAIN_OK;
}

louvain_status louvain_coarsen(louvain_graph_t g, int64_t *n_new_out)
{
    louvain_status s = check_handle(g);
    if (s) return s;
    int64_t n_new = 0;
    if ((s = coarsen_current(g, g->comm_prev, n_new))) return s;
    if (n_new_out) *n_new_out = n_new;
    return LOUVAIN_OK;
}

louvain_status louvain_run(louvain_graph_t g, const louvain_params *p, int32_t *labels_out, uint32_t labels_on_device,
                           louvain_result *out)
{
    louvain_status s = check_handle(g);
    if (s) return s;
    if ((s = check_params(g, p))) return s;
    const auto t_start = std::chrono::steady_clock::now();
    g->phases.clear();
    g->iters.clear();
    g->swept_entries = 0;
    g->lookahead_entries = 0;
    if ((s = reset_level0(g))) return s;
    louvain_result res;
    std::memset(&res, 0, sizeof(res));
    res.n_orig = g->n0;
    double ms_vf = 0, ms_color = 0, ms_sweep = 0, ms_coarsen = 0;
    const i128 D = (i128)g->two_m * g->two_m;
    i128 N_final = 0, N0 = 0;
    int64_t K = g->n0;
    if (g->two_m > 0) {
        if (p->vf) {
            const auto t0 = std::chrono::steady_clock::now();
            if ((s = vertex_following(g, p->vf, [](int64_t, int64_t) { return LOUVAIN_OK; }, &res.vf_rounds)))
                return s;
            ms_vf = ms_since(t0);
        }
        res.n_vf = g->cur.n;
        i128 s2;
        if ((s = sum_sq(g, g->k, g->cur.n, s2))) return s;
        N0 = (i128)g->two_m * g->self - s2;
        i128 Q_prev = N0;
        bool still_coloring = p->color != 0;
        for (int ph_idx = 1;; ++ph_idx) {
            const bool colored = still_coloring && g->cur.n >= p->color_cutoff;
            const louvain_ratio th = colored ? p->theta_color : p->theta_final;
            louvain_phase_stats ph;
            std::memset(&ph, 0, sizeof(ph));
            ph.n = g->cur.n;
            ph.nnz = g->cur.nnz;
            ph.colored = colored;
            ph.first_iter = (int64_t)g->iters.size();
            auto t0 = std::chrono::steady_clock::now();
            if (colored) {
                if ((s = do_color(g, p->color_seed))) return s;
                if (p->color_balance && (s = do_balance(g, p->color_seed, nullptr))) return s;
                ph.num_colors = g->num_colors;
            }
            ph.ms_color = ms_since(t0);
            ms_color += ph.ms_color;
            t0 = std::chrono::steady_clock::now();
            if ((s = build_bins(g, colored))) return s;
            // the phase starts from singletons: its Q_0 is the previous phase's Q
            if (colored) s = run_phase_colored(g, p, th, ph, Q_prev);
            else s = run_phase_plain(g, p, th, ph, Q_prev);
            if (s) return s;
            ph.ms_sweep = ms_since(t0);
            ms_sweep += ph.ms_sweep;
            const i128 Np = (i128)(((u128)(uint64_t)ph.q_num.hi << 64) | (u128)ph.q_num.lo);
            t0 = std::chrono::steady_clock::now();
            const int64_t n_before = g->cur.n;
            int64_t n_after = 0;
            if ((s = coarsen_current(g, g->comm_prev, n_after))) return s;
            ph.ms_coarsen = ms_since(t0);
            ms_coarsen += ph.ms_coarsen;
            g->phases.push_back(ph);
            bool stop;
            if (colored) {
                if (n_after < p->color_cutoff || n_after == n_before || p->color_first_phase_only ||
                    below_threshold(Np, Q_prev, D, p->theta_color, 0))
                    still_coloring = false;
                stop = ph_idx >= p->max_phases;
            } else {
                stop = n_after == n_before || ph_idx >= p->max_phases ||
                       below_threshold(Np, Q_prev, D, p->theta_final, 0);
            }
            Q_prev = Np;
            if (stop) break;
        }
        N_final = Q_prev;
        K = g->cur.n;
    } else {
        res.n_vf = g->n0;
    }
    if (labels_out && g->n0)
        if ((s = copy_out(g, labels_out, g->orig_map, g->n0 * sizeof(int32_t), labels_on_device))) return s;
    if ((s = sync(g))) return s;
    if (out) {
        res.num_communities = K;
        res.phases = (int64_t)g->phases.size();
        res.iterations = (int64_t)g->iters.size();
        res.q_num = to_abi(g->two_m > 0 ? N_final : (i128)0);
        res.q_den = to_abi(g->two_m > 0 ? D : (i128)1);
        res.q0_num = to_abi(N0);
        res.q = g->two_m > 0 ? exact_ratio(N_final, D) : 0.0;
        res.sweep_entries = g->swept_entries - g->lookahead_entries;
        res.lookahead_entries = g->lookahead_entries;
        res.ms_total = ms_since(t_start);
        res.ms_vf = ms_vf;
        res.ms_color = ms_color;
        res.ms_sweep = ms_sweep;
        res.ms_coarsen = ms_coarsen;
        res.phase = g->phases.data();
        res.iter = g->iters.data();
        *out = res;
    }
    return LOUVAIN_OK;
}

louvain_status louvain_get_info(louvain_graph_t g, int64_t *out)
{
    louvain_status s = check_handle(g);
    if (s) return s;
    if (!out) return fail(g, LOUVAIN_E_INVALID_ARG, "out is NULL");
    out[0] = g->cur.n;
    out[1] = g->cur.nnz;
    out[2] = g->two_m;
    out[3] = g->n0;
    out[4] = g->colored ? g->num_colors : 0;
    out[5] = g->cur.wk;
    out[6] = g->kmax;
    out[7] = g->level;
    return LOUVAIN_OK;
}

louvain_status louvain_get_state(louvain_graph_t g, int32_t *comm, int64_t *a, int32_t *size, int64_t *k,
                                 uint32_t on_device)
{
    louvain_status s = check_handle(g);
    if (s) return s;
    const int64_t n = g->cur.n;
    if ((s = copy_out(g, comm, g->comm_prev, n * sizeof(int32_t), on_device))) return s;
    if ((s = copy_out(g, a, g->a, n * sizeof(int64_t), on_device))) return s;
    if ((s = copy_out(g, size, g->size, n * sizeof(int32_t), on_device))) return s;
    return copy_out(g, k, g->k, n * sizeof(int64_t), on_device);
}

louvain_status louvain_get_graph(louvain_graph_t g, int64_t *offsets, int32_t *cols, int64_t *weights,
                                 uint32_t on_device)
{
    louvain_status s = check_handle(g);
    if (s) return s;
    if ((s = copy_out(g, offsets, g->cur.off, (g->cur.n + 1) * sizeof(int64_t), on_device))) return s;
    if ((s = copy_out(g, cols, g->cur.col, g->cur.nnz * sizeof(int32_t), on_device))) return s;
    if (weights && g->cur.nnz) {
        if (g->cur.wk == lv::W_I64) return copy_out(g, weights, g->cur.w, g->cur.nnz * sizeof(int64_t), on_device);
        lv::weights_i64(g->cur, (int64_t *)g->vals, g->st);
        return copy_out(g, weights, g->vals, g->cur.nnz * sizeof(int64_t), on_device);
    }
    return LOUVAIN_OK;
}

louvain_status louvain_get_colors(louvain_graph_t g, int32_t *color, uint32_t on_device)
{
    louvain_status s = check_handle(g);
    if (s) return s;
    if (!g->colored) return fail(g, LOUVAIN_E_STATE, "the current graph is not colored");
    return copy_out(g, color, g->color, g->cur.n * sizeof(int32_t), on_device);
}

louvain_status louvain_get_map(louvain_graph_t g, int32_t *orig_map, uint32_t on_device)
{
    louvain_status s = check_handle(g);
    if (s) return s;
    return copy_out(g, orig_map, g->orig_map, g->n0 * sizeof(int32_t), on_device);
}

louvain_status louvain_profile(louvain_graph_t g, int32_t enable)
{
    louvain_status s = check_handle(g);
    if (s) return s;
    if ((s = sync(g))) return s;
    prof_collect(g, nullptr, 0);
    g->prof = enable != 0;
    for (auto &r : g->recs) {
        r.launches = 0;
        r.ms = r.bytes = r.entries = 0;
    }
    return LOUVAIN_OK;
}

louvain_status louvain_profile_get(louvain_graph_t g, int32_t idx, const char **name, int64_t *launches,
                                   double *total_ms, double *bytes, double *entries)
{
    if (!g) return LOUVAIN_E_INVALID_ARG;
    if (idx < 0 || idx >= (int32_t)g->recs.size()) return LOUVAIN_E_INVALID_ARG;
    const ProfRec &r = g->recs[idx];
    if (name) *name = r.name;
    if (launches) *launches = r.launches;
    if (total_ms) *total_ms = r.ms;
    if (bytes) *bytes = r.bytes;
    if (entries) *entries = r.entries;
    return LOUVAIN_OK;
}



} // extern "C"

// ===========================================================================
// Allocation-free run.  Every buffer of the run is carved from `scratch`, a
// fixed device array of this file (one copy per GPU, held until the process
// ends), so the call makes no device allocation.  In host code `scratch`
// names a host-side stand-in: its device address is taken once per device
// with hipGetSymbolAddress and only that address is ever used.
// ===========================================================================
namespace {

constexpr size_t kScratchBytes = (size_t)LOUVAIN_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, char *> g_scratch_ptr; // device -> device address of its copy of scratch

// the current device's copy of scratch, looked up once per device
louvain_status scratch_address(int dev, char **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return LOUVAIN_OK;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return fail(nullptr, LOUVAIN_E_HIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = (char *)p;
    *out = (char *)p;
    return LOUVAIN_OK;
}

// phase and iteration records of the last allocation-free run of this thread
thread_local std::vector<louvain_phase_stats> t_noalloc_phases;
thread_local std::vector<louvain_iter_stats> t_noalloc_iters;

} // namespace

extern "C" {

louvain_status louvain_run_noalloc(int64_t n, int64_t nnz, const int64_t *offsets, const int32_t *cols,
                                   const int32_t *weights, uint32_t flags, const louvain_params *params,
                                   int32_t *labels_out, void *hip_stream, louvain_result *out)
{
    g_init_error.clear();
    if (flags & ~LOUVAIN_VALIDATE) return fail(nullptr, LOUVAIN_E_INVALID_ARG, "only LOUVAIN_VALIDATE is accepted");
    flags |= LOUVAIN_DEVICE_PTRS;
    louvain_status s = check_csr_args(n, nnz, offsets, cols, flags);
    if (s) return s;
    // the buffers the handle needs, measured without carving anything
    G probe;
    probe.count_only = true;
    (void)alloc_buffers(&probe, n, nnz, weights != nullptr);
    if (probe.arena_used > kScratchBytes)
        return fail(nullptr, LOUVAIN_E_INVALID_ARG,
                    "graph too large for louvain_run_noalloc: its buffers need " + std::to_string(probe.arena_used) +
                        " bytes of the " + std::to_string(kScratchBytes) + "-byte scratch");
    G g;
    g.st = (hipStream_t)hip_stream;
    if (const hipError_t e = hipGetDevice(&g.dev))
        return fail(nullptr, LOUVAIN_E_HIP, std::string("hipGetDevice failed: ") + hipGetErrorString(e));
    if ((s = scratch_address(g.dev, &g.arena))) return s;
    g.arena_cap = kScratchBytes;
    // no HIP graphs, no timing events, default lanes: nothing but kernels and copies
    g.graphs_ok = false;
    g.tune = false;
    auto done = [&](louvain_status st) {
        if (st) g_init_error = g.err;
        release_all(&g);
        return st;
    };
    if ((s = alloc_buffers(&g, n, nnz, weights != nullptr))) return done(s);
    if ((s = ingest(&g, n, nnz, offsets, cols, weights, flags))) return done(s);
    louvain_result res;
    if ((s = louvain_run(&g, params, labels_out, 1, &res))) return done(s);
    t_noalloc_phases = g.phases;
    t_noalloc_iters = g.iters;
    res.phase = t_noalloc_phases.data();
    res.iter = t_noalloc_iters.data();
    if (out) *out = res;
    return done(LOUVAIN_OK);
}

} // extern "C"

// ===========================================================================
// Batched form: many independent graphs in one disjoint-union CSR.  Every
// launch covers all graphs; each graph keeps its own iteration and phase
// decisions (the rules of louvain_run, applied per graph on the host from
// per-graph sweep statistics), so every graph's result is the one it gets
// alone.  Coloring is not available in this form.
// ===========================================================================
struct louvain_batch_s {
    G *g = nullptr;
    int32_t ng = 0;
    std::string err;
    std::vector<int64_t> goff0, goff; // input / current graph offsets (host)
    int64_t *goff_d = nullptr, *goff_tmp = nullptr, *gsum = nullptr, *gstats = nullptr, *two_m_d = nullptr,
            *idx_d = nullptr, *gath = nullptr;
    int32_t *gid0 = nullptr, *gid = nullptr, *active_d = nullptr, *keep_d = nullptr, *labels_tmp = nullptr;
    std::vector<int64_t> two_m;
    struct Run {
        std::vector<louvain_phase_stats> phases;
        std::vector<louvain_iter_stats> iters;
        int64_t n = 0, nnz = 0, K = 0, n_vf = 0;
        i128 N = 0, N0 = 0, Q_prev = 0;
        bool finished = false;
        // current phase
        bool sweeping = false;
        std::vector<i128> S2, Nt;
        int t_end = 0, hit = 0, undone = 0;
    };
    std::vector<Run> runs;
};

namespace {

typedef louvain_batch_s B;

louvain_status bfail(B *b, louvain_status s, const std::string &m)
{
    b->err = m;
    return s;
}

// current graph offsets (device goff_d) -> host goff; graph ids of the current level
louvain_status batch_refresh_ids(B *b)
{
    G *g = b->g;
    HIPCHK(g, hipMemcpyAsync(b->goff.data(), b->goff_d, (b->ng + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, g->st));
    lv::graph_ids(b->goff_d, b->ng, g->cur.n, b->gid, g->st);
    return sync(g);
}

// after coarsen_current: new graph offsets from the renumbering
louvain_status batch_after_coarsen(B *b, int64_t n_before, int64_t n_after)
{
    G *g = b->g;
    lv::new_graph_offsets(b->goff_d, b->ng, n_before, g->new_id, n_after, b->goff_tmp, g->st);
    std::swap(b->goff_d, b->goff_tmp);
    return batch_refresh_ids(b);
}

// per-graph sums of x (and self-loops if with_self) into host vectors
louvain_status batch_sums(B *b, const int64_t *x, bool with_self, std::vector<i128> &sq, std::vector<int64_t> *sum,
                          std::vector<int64_t> *self)
{
    G *g = b->g;
    lv::graph_sums(g->cur, with_self, x, b->gid, b->ng, b->gsum, g->st);
    std::vector<int64_t> h(4 * (size_t)b->ng);
    if (b->ng) HIPCHK(g, hipMemcpyAsync(h.data(), b->gsum, h.size() * sizeof(int64_t), hipMemcpyDeviceToHost, g->st));
    louvain_status s = sync(g);
    if (s) return s;
    sq.resize(b->ng);
    if (sum) sum->resize(b->ng);
    if (self) self->resize(b->ng);
    for (int32_t i = 0; i < b->ng; ++i) {
        sq[i] = (i128)(((u128)(uint64_t)h[4 * i + 2] << 64) | (u128)(uint64_t)h[4 * i + 1]);
        if (sum) (*sum)[i] = h[4 * i];
        if (self) (*self)[i] = h[4 * i + 3];
    }
    return LOUVAIN_OK;
}

// CSR entries of every graph of the current level
louvain_status batch_nnz(B *b, std::vector<int64_t> &nnz)
{
    G *g = b->g;
    lv::gather_i64(g->cur.off, b->goff_d, b->ng + 1, b->gath, g->st);
    std::vector<int64_t> h(b->ng + 1);
    HIPCHK(g, hipMemcpyAsync(h.data(), b->gath, (b->ng + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, g->st));
    louvain_status s = sync(g);
    if (s) return s;
    nnz.resize(b->ng);
    for (int32_t i = 0; i < b->ng; ++i) nnz[i] = h[i + 1] - h[i];
    return LOUVAIN_OK;
}

} // namespace

extern "C" {

louvain_status louvain_batch_init(int32_t num_graphs, const int64_t *graph_off, int64_t nnz, const int64_t *offsets,
                                  const int32_t *cols, const int32_t *weights, uint32_t flags, void *hip_stream,
                                  louvain_batch_t *out)
{
    g_init_error.clear();
    if (!out) return fail(nullptr, LOUVAIN_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (num_graphs < 0 || !graph_off) return fail(nullptr, LOUVAIN_E_INVALID_ARG, "bad graph offsets");
    if (graph_off[0] != 0) return fail(nullptr, LOUVAIN_E_BAD_CSR, "graph_off[0] must be 0");
    for (int32_t i = 0; i < num_graphs; ++i)
        if (graph_off[i + 1] < graph_off[i]) return fail(nullptr, LOUVAIN_E_BAD_CSR, "graph offsets not monotone");
    const int64_t n = graph_off[num_graphs];
    louvain_graph_t g = nullptr;
    louvain_status s = louvain_init_csr(n, nnz, offsets, cols, weights, flags, hip_stream, &g);
    if (s) return s;
    B *b = new B();
    b->g = g;
    b->ng = num_graphs;
    b->goff0.assign(graph_off, graph_off + num_graphs + 1);
    b->goff = b->goff0;
    auto bail = [&](louvain_status st) {
        g_init_error = g->err.empty() ? b->err : g->err;
        louvain_destroy(g);
        delete b;
        return st;
    };
    const int64_t ng1 = num_graphs + 1;
    if ((s = alloc(g, &b->goff_d, ng1)) || (s = alloc(g, &b->goff_tmp, ng1)) || (s = alloc(g, &b->gsum, 4 * ng1)) ||
        (s = alloc(g, &b->gstats, 8 * ng1)) || (s = alloc(g, &b->two_m_d, ng1)) || (s = alloc(g, &b->gath, ng1)) ||
        (s = alloc(g, &b->gid0, n)) || (s = alloc(g, &b->gid, n)) || (s = alloc(g, &b->active_d, ng1)) ||
        (s = alloc(g, &b->keep_d, ng1)) || (s = alloc(g, &b->labels_tmp, n)))
        return bail(s);
    if (hipMemcpyAsync(b->goff_d, graph_off, ng1 * sizeof(int64_t), hipMemcpyHostToDevice, g->st) != hipSuccess)
        return bail(LOUVAIN_E_HIP);
    lv::graph_ids(b->goff_d, num_graphs, n, b->gid0, g->st);
    // every edge must stay inside its graph
    int32_t code = 0;
    lv::fill<int32_t>(g->vflag, 0, 1, g->st);
    lv::cross_edges(g->cur, b->gid0, g->vflag, g->st);
    if (hipMemcpyAsync(&code, g->vflag, sizeof(code), hipMemcpyDeviceToHost, g->st) != hipSuccess ||
        hipStreamSynchronize(g->st) != hipSuccess)
        return bail(LOUVAIN_E_HIP);
    if (code) {
        g->err = "invalid batch: an edge joins two different graphs";
        return bail(LOUVAIN_E_BAD_CSR);
    }
    *out = b;
    return LOUVAIN_OK;
}

void louvain_batch_destroy(louvain_batch_t b)
{
    if (!b) return;
    louvain_destroy(b->g);
    delete b;
}

const char *louvain_batch_last_error(louvain_batch_t b)
{
    if (!b) return g_init_error.c_str();
    return b->err.empty() ? b->g->err.c_str() : b->err.c_str();
}

louvain_status louvain_batch_init_graphs(int32_t num_graphs, const int64_t *n, const int64_t *nnz,
                                         const int64_t *const *offsets, const int32_t *const *cols,
                                         const int32_t *const *weights, uint32_t flags, void *hip_stream,
                                         louvain_batch_t *out)
{
    g_init_error.clear();
    if (!out) return fail(nullptr, LOUVAIN_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (num_graphs < 0 || (num_graphs > 0 && (!n || !nnz || !offsets || !cols)))
        return fail(nullptr, LOUVAIN_E_INVALID_ARG, "bad graph arrays");
    if (flags & ~LOUVAIN_VALIDATE) return fail(nullptr, LOUVAIN_E_INVALID_ARG, "host arrays only (VALIDATE allowed)");
    std::vector<int64_t> goff(num_graphs + 1, 0), eoff(num_graphs + 1, 0);
    bool weighted = false;
    for (int32_t i = 0; i < num_graphs; ++i) {
        if (n[i] < 0 || nnz[i] < 0 || !offsets[i] || (nnz[i] > 0 && !cols[i]))
            return fail(nullptr, LOUVAIN_E_INVALID_ARG, "bad arrays of graph " + std::to_string(i));
        if (offsets[i][0] != 0 || offsets[i][n[i]] != nnz[i])
            return fail(nullptr, LOUVAIN_E_BAD_CSR, "offsets of graph " + std::to_string(i) + " do not span [0, nnz]");
        goff[i + 1] = goff[i] + n[i];
        eoff[i + 1] = eoff[i] + nnz[i];
        weighted |= weights && weights[i];
    }
    const int64_t N = goff[num_graphs], E = eoff[num_graphs];
    if (N >= ((int64_t)1 << 31) - 1) return fail(nullptr, LOUVAIN_E_INVALID_ARG, "n must be below 2^31 - 1");
    hipStream_t st = (hipStream_t)hip_stream;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(nullptr, LOUVAIN_E_HIP, "no device");
    // staging buffers: the union CSR, then the graph and entry offsets
    const size_t b_off = (N + 1) * sizeof(int64_t), b_col = (E > 0 ? E : 1) * sizeof(int32_t);
    const size_t b_idx = 2 * (num_graphs + 1) * sizeof(int64_t);
    void *p_off = nullptr, *p_col = nullptr, *p_w = nullptr, *p_idx = nullptr;
    auto release = [&]() {
        if (st) (void)hipStreamSynchronize(st);
        else (void)hipDeviceSynchronize();
        pool().put(p_off, b_off, dev);
        pool().put(p_col, b_col, dev);
        if (p_w) pool().put(p_w, b_col, dev);
        pool().put(p_idx, b_idx, dev);
    };
    if (pool().get(&p_off, b_off, dev) != hipSuccess || pool().get(&p_col, b_col, dev) != hipSuccess ||
        (weighted && pool().get(&p_w, b_col, dev) != hipSuccess) || pool().get(&p_idx, b_idx, dev) != hipSuccess) {
        (void)hipGetLastError();
        release();
        return fail(nullptr, LOUVAIN_E_OOM, "staging allocation failed");
    }
    int64_t *d_off = (int64_t *)p_off, *d_idx = (int64_t *)p_idx;
    int32_t *d_col = (int32_t *)p_col, *d_w = (int32_t *)p_w;
    bool ok = true;
    for (int32_t i = 0; i < num_graphs && ok; ++i) {
        if (n[i]) ok &= hipMemcpyAsync(d_off + goff[i], offsets[i], n[i] * sizeof(int64_t), hipMemcpyHostToDevice, st) == hipSuccess;
        if (nnz[i]) {
            ok &= hipMemcpyAsync(d_col + eoff[i], cols[i], nnz[i] * sizeof(int32_t), hipMemcpyHostToDevice, st) == hipSuccess;
            if (weighted) {
                if (weights[i])
                    ok &= hipMemcpyAsync(d_w + eoff[i], weights[i], nnz[i] * sizeof(int32_t), hipMemcpyHostToDevice,
                                         st) == hipSuccess;
                else
                    lv::fill<int32_t>(d_w + eoff[i], 1, nnz[i], st);
            }
        }
    }
    ok = ok && hipMemcpyAsync(d_idx, goff.data(), (num_graphs + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(d_idx + num_graphs + 1, eoff.data(), (num_graphs + 1) * sizeof(int64_t), hipMemcpyHostToDevice,
                              st) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        release();
        return fail(nullptr, LOUVAIN_E_HIP, "copy of the graphs failed");
    }
    lv::batch_fixup(d_off, N, d_col, E, d_idx, d_idx + num_graphs + 1, num_graphs, st);
    // the union's last offset is E: graph i's offsets were copied without their final entry
    lv::fill<int64_t>(d_off + N, E, 1, st);
    const louvain_status s = louvain_batch_init(num_graphs, goff.data(), E, d_off, d_col, weighted ? d_w : nullptr,
                                                flags | LOUVAIN_DEVICE_PTRS, hip_stream, out);
    release();
    return s;
}

louvain_status louvain_batch_run(louvain_batch_t b, const louvain_params *p, int32_t *labels_out,
                                 uint32_t labels_on_device, louvain_graph_result *results)
{
    if (!b) return LOUVAIN_E_INVALID_ARG;
    b->err.clear();
    G *g = b->g;
    louvain_status s = check_handle(g);
    if (s) return s;
    if ((s = check_params(g, p))) return s;
    if (p->color) return bfail(b, LOUVAIN_E_INVALID_ARG, "the batched form runs uncolored phases (color must be 0)");
    const int32_t ng = b->ng;
    g->phases.clear();
    g->iters.clear();
    if ((s = reset_level0(g))) return s;
    b->goff = b->goff0;
    HIPCHK(g, hipMemcpyAsync(b->goff_d, b->goff0.data(), (ng + 1) * sizeof(int64_t), hipMemcpyHostToDevice, g->st));
    if ((s = batch_refresh_ids(b))) return s;
    b->runs.assign(ng, B::Run());
    std::vector<i128> sq;
    std::vector<int64_t> sum, self, nnz;
    if ((s = batch_sums(b, g->k, true, sq, &sum, &self))) return s;
    b->two_m = sum;
    HIPCHK(g, hipMemcpyAsync(b->two_m_d, b->two_m.data(), ng * sizeof(int64_t), hipMemcpyHostToDevice, g->st));
    if ((s = batch_nnz(b, nnz))) return s;
    for (int32_t i = 0; i < ng; ++i) {
        B::Run &r = b->runs[i];
        r.n = b->goff[i + 1] - b->goff[i];
        r.nnz = nnz[i];
        r.finished = b->two_m[i] == 0;
        r.K = r.n;
        r.n_vf = r.n;
    }
    g->b_gid = b->gid;
    g->b_two_m = b->two_m_d;
    g->b_active = b->active_d;
    g->b_gstats = b->gstats;
    struct Unbind {
        G *g;
        ~Unbind() { g->b_gid = nullptr; g->b_two_m = nullptr; g->b_active = nullptr; g->b_gstats = nullptr; }
    } unbind{g};

    if (p->vf && g->two_m > 0) {
        // chain rounds take each graph's own 2m (b_gid, b_two_m are bound)
        if ((s = vertex_following(g, p->vf, [&](int64_t n0, int64_t nv) { return batch_after_coarsen(b, n0, nv); },
                                  nullptr)))
            return s;
    }
    if ((s = batch_sums(b, g->k, true, sq, nullptr, &self))) return s;
    for (int32_t i = 0; i < ng; ++i) {
        B::Run &r = b->runs[i];
        r.n_vf = b->goff[i + 1] - b->goff[i];
        if (!r.finished) r.N0 = r.Q_prev = (i128)b->two_m[i] * self[i] - sq[i];
    }
    std::vector<int32_t> active(ng + 1, 0), keep(ng + 1, 0);
    std::vector<int64_t> gst(8 * (size_t)(ng + 1));
    for (int ph_idx = 1;; ++ph_idx) {
        bool any = false;
        for (auto &r : b->runs) any |= !r.finished;
        if (!any) break;
        if ((s = batch_nnz(b, nnz))) return s;
        // phase start: every graph from singletons; its Q_0 is its previous phase's Q
        for (int32_t i = 0; i < ng; ++i) {
            B::Run &r = b->runs[i];
            active[i] = !r.finished;
            r.sweeping = !r.finished;
            if (r.finished) continue;
            louvain_phase_stats ph;
            std::memset(&ph, 0, sizeof(ph));
            ph.n = b->goff[i + 1] - b->goff[i];
            ph.nnz = nnz[i];
            ph.first_iter = (int64_t)r.iters.size();
            r.phases.push_back(ph);
            r.S2.assign(1, sq[i]);
            r.Nt.assign(1, r.Q_prev);
            r.t_end = 0;
            r.hit = 0;
            r.undone = 0;
        }
        HIPCHK(g, hipMemcpyAsync(b->active_d, active.data(), ng * sizeof(int32_t), hipMemcpyHostToDevice, g->st));
        // the bins hold only the vertices of sweeping graphs; they are rebuilt
        // whenever that set has halved
        auto active_vertices = [&]() {
            int64_t v = 0;
            for (int32_t i = 0; i < ng; ++i)
                if (active[i]) v += b->goff[i + 1] - b->goff[i];
            return v;
        };
        if ((s = build_bins(g, false, true))) return s;
        int64_t binned = active_vertices();
        for (int sidx = 1;; ++sidx) {
            if ((s = run_stage(g, g->stage_batch, [&]() {
                     lv::fill<int64_t>(b->gstats, 0, 8 * (int64_t)ng, g->st);
                     sweep_group(g, 0, p->singlet_rule);
                 })))
                return s;
            if (ng) HIPCHK(g, hipMemcpyAsync(gst.data(), b->gstats, 8 * ng * sizeof(int64_t), hipMemcpyDeviceToHost, g->st));
            if ((s = sync(g))) return s;
            prof_collect(g, nullptr, 0);
            bool any_keep = false;
            for (int32_t i = 0; i < ng; ++i) {
                keep[i] = 0;
                B::Run &r = b->runs[i];
                if (!r.sweeping) continue;
                const int64_t moves = gst[8 * i + 0], sigma = gst[8 * i + 1];
                const i128 D = (i128)b->two_m[i] * b->two_m[i];
                const louvain_ratio th = p->theta_final;
                g->swept_entries += gst[8 * i + 4];
                if (sidx >= 2) {
                    r.Nt[sidx - 1] = (i128)b->two_m[i] * sigma - r.S2[sidx - 1];
                    r.iters.back().q_num = to_abi(r.Nt[sidx - 1]);
                    const int64_t look = gst[8 * i + 4];
                    if (r.Nt[sidx - 1] < r.Nt[sidx - 2]) { // a loss: undone, the phase ends (Sec. 5.1)
                        g->lookahead_entries += look;
                        keep[i] = 2;
                        r.undone = 1;
                        r.t_end = sidx - 1;
                        r.sweeping = false;
                        continue;
                    }
                    if (sidx - 1 >= 2 && below_threshold(r.Nt[sidx - 1], r.Nt[sidx - 2], D, th, p->threshold_mode)) {
                        g->lookahead_entries += look;
                        r.t_end = sidx - 1;
                        r.sweeping = false;
                        continue;
                    }
                    if (sidx - 1 >= p->max_iter) {
                        g->lookahead_entries += look;
                        r.hit = 1;
                        r.t_end = sidx - 1;
                        r.sweeping = false;
                        continue;
                    }
                }
                louvain_iter_stats rec{};
                rec.moves = moves;
                rec.pairs = gst[8 * i + 3];
                rec.entries = gst[8 * i + 4];
                r.iters.push_back(rec);
                r.Nt.push_back(0);
                r.S2.push_back(0);
                if (moves == 0) {
                    r.Nt[sidx] = r.Nt[sidx - 1];
                    r.S2[sidx] = r.S2[sidx - 1];
                    r.iters.back().q_num = to_abi(r.Nt[sidx]);
                    r.t_end = sidx;
                    r.sweeping = false;
                    continue;
                }
                keep[i] = 1;
                any_keep = true;
            }
            HIPCHK(g, hipMemcpyAsync(b->keep_d, keep.data(), ng * sizeof(int32_t), hipMemcpyHostToDevice, g->st));
            {
                ProfScope ps(g, PR_COMMIT, 8.0 * (double)g->cur.n, 0);
                lv::commit_graphs(g->cur.n, g->comm_prev, g->comm_next, g->comm_save, g->k, g->a, g->size, b->gid,
                                  b->keep_d, g->st);
                g->singleton = false;
            }
            if (any_keep) {
                std::vector<i128> s2;
                if ((s = batch_sums(b, g->a, false, s2, nullptr, nullptr))) return s;
                for (int32_t i = 0; i < ng; ++i)
                    if (keep[i] == 1) b->runs[i].S2[sidx] = s2[i];
            }
            bool still = false;
            for (int32_t i = 0; i < ng; ++i) {
                active[i] = b->runs[i].sweeping;
                still |= b->runs[i].sweeping;
            }
            if (!still) break;
            HIPCHK(g, hipMemcpyAsync(b->active_d, active.data(), ng * sizeof(int32_t), hipMemcpyHostToDevice, g->st));
            const int64_t now = active_vertices();
            if (2 * now < binned) {
                if ((s = build_bins(g, false, true))) return s;
                binned = now;
            }
        }
        if ((s = sync(g))) return s;
        // rebuild every graph (a finished graph sits at singletons: an identity rebuild)
        const int64_t n_before_all = g->cur.n;
        std::vector<int64_t> n_before(ng);
        for (int32_t i = 0; i < ng; ++i) n_before[i] = b->goff[i + 1] - b->goff[i];
        int64_t n_after_all = 0;
        if ((s = coarsen_current(g, g->comm_prev, n_after_all))) return s;
        if ((s = batch_after_coarsen(b, n_before_all, n_after_all))) return s;
        if ((s = batch_sums(b, g->k, true, sq, nullptr, nullptr))) return s;
        for (int32_t i = 0; i < ng; ++i) {
            B::Run &r = b->runs[i];
            if (r.finished) continue;
            louvain_phase_stats &ph = r.phases.back();
            ph.iterations = r.t_end;
            ph.hit_max_iter = r.hit;
            ph.loss_undone = r.undone;
            const i128 Np = r.undone ? r.Nt[r.t_end - 1] : r.Nt[r.t_end];
            ph.q_num = to_abi(Np);
            const int64_t n_after = b->goff[i + 1] - b->goff[i];
            const i128 D = (i128)b->two_m[i] * b->two_m[i];
            const bool stop = n_after == n_before[i] || ph_idx >= p->max_phases ||
                              below_threshold(Np, r.Q_prev, D, p->theta_final, 0);
            r.Q_prev = Np;
            if (stop) r.finished = true;
        }
    }
    // labels local to each graph
    if (labels_out && g->n0) {
        lv::local_labels(g->orig_map, b->gid0, g->n0, b->goff_d, b->labels_tmp, g->st);
        if ((s = copy_out(g, labels_out, b->labels_tmp, g->n0 * sizeof(int32_t), labels_on_device))) return s;
    }
    if ((s = sync(g))) return s;
    if (results) {
        for (int32_t i = 0; i < ng; ++i) {
            B::Run &r = b->runs[i];
            louvain_graph_result &o = results[i];
            std::memset(&o, 0, sizeof(o));
            o.n = b->goff0[i + 1] - b->goff0[i];
            o.nnz = r.nnz;
            o.num_communities = b->goff[i + 1] - b->goff[i];
            o.phases = (int64_t)r.phases.size();
            o.iterations = (int64_t)r.iters.size();
            o.n_vf = r.n_vf;
            const bool edges = b->two_m[i] > 0;
            const i128 D = edges ? (i128)b->two_m[i] * b->two_m[i] : (i128)1;
            o.q_num = to_abi(edges ? r.Q_prev : (i128)0);
            o.q_den = to_abi(D);
            o.q0_num = to_abi(edges ? r.N0 : (i128)0);
            o.q = edges ? exact_ratio(r.Q_prev, D) : 0.0;
        }
    }
    return LOUVAIN_OK;
}

louvain_status louvain_batch_graph_stats(louvain_batch_t b, int32_t graph, const louvain_phase_stats **phases,
                                         int64_t *num_phases, const louvain_iter_stats **iters, int64_t *num_iters)
{
    if (!b || graph < 0 || graph >= b->ng || graph >= (int32_t)b->runs.size()) return LOUVAIN_E_INVALID_ARG;
    const B::Run &r = b->runs[graph];
    if (phases) *phases = r.phases.data();
    if (num_phases) *num_phases = (int64_t)r.phases.size();
    if (iters) *iters = r.iters.data();
    if (num_iters) *num_iters = (int64_t)r.iters.size();
    return LOUVAIN_OK;
}

} // extern "C"
