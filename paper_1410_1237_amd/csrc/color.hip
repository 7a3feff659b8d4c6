// Distance-1 coloring (Sec. 5.2) by Jones-Plassmann rounds with hashed
// priorities pi(v) = SplitMix64 finalizer((seed << 32) ^ v) (Steele, Lea,
// Flood 2014).  Priorities are a bijection of v, so every vertex has a
// strict rank; a vertex is coloured once all its higher-priority neighbours
// are, with the smallest colour none of them uses.  The result is therefore
// exactly the greedy colouring in descending priority, for any schedule.
//
// Instead of re-testing every uncoloured vertex each round, each vertex
// keeps the count of its uncoloured higher-priority neighbours; colouring a
// vertex decrements its lower-priority neighbours and the ones reaching zero
// form the next round's frontier, so every row is scanned a bounded number
// of times.  Rows longer than LIGHT_MAX are coloured by a whole workgroup
// with an LDS bitmap of used colours.
#include "lv.h"

namespace lv {

constexpr int64_t LIGHT_MAX = 256;
constexpr int BITMAP_WORDS = 1024; // 32,768 colours per window

__device__ __forceinline__ uint64_t jp_priority(uint64_t seed, int64_t v)
{
    uint64_t z = (seed << 32) ^ (uint64_t)v;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// cnt[v] = number of neighbours u != v with pi(u) > pi(v)
__global__ __launch_bounds__(BLOCK) void k_jp_count(Csr g, uint64_t seed, int32_t *cnt)
{
    __shared__ int64_t s_off[ROWCAP + 1];
    __shared__ int64_t s_meta[2];
    const int64_t e0 = (int64_t)blockIdx.x * ETILE;
    const int64_t e1 = min(e0 + ETILE, g.nnz) - 1;
    TileRows t = tile_rows(g.off, g.n, e0, e1, s_off, s_meta);
    for (int r = 0; r < EITEMS; ++r) {
        const int64_t e = e0 + r * BLOCK + threadIdx.x;
        if (e > e1) break;
        const int64_t v = tile_row(t, g.off, s_off, e);
        const int32_t u = g.col[e];
        if (u != v && jp_priority(seed, u) > jp_priority(seed, v)) atomicAdd(&cnt[v], 1);
    }
}

__global__ __launch_bounds__(BLOCK) void k_jp_start(const int32_t *cnt, int64_t n, int32_t *color, int32_t *front,
                                                    int32_t *counters)
{
    for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * BLOCK) {
        color[v] = -1;
        if (cnt[v] == 0) front[atomicAdd(&counters[0], 1)] = (int32_t)v;
    }
}

// decrement lower-priority neighbours of v; append the ones that become ready
__device__ __forceinline__ void jp_release(const Csr &g, uint64_t seed, int64_t v, uint64_t pv, int64_t e_begin,
                                           int64_t e_end, int stride, int32_t *cnt, int32_t *next,
                                           int32_t *next_count)
{
    for (int64_t e = e_begin; e < e_end; e += stride) {
        const int32_t u = g.col[e];
        if (u != v && jp_priority(seed, u) < pv)
            if (atomicSub(&cnt[u], 1) == 1) next[atomicAdd(next_count, 1)] = u;
    }
}

// light rows: one thread per frontier vertex; heavy rows are deferred to k_jp_heavy
__global__ __launch_bounds__(BLOCK) void k_jp_light(Csr g, uint64_t seed, const int32_t *front, const int32_t *counters,
                                                    int32_t *color, int32_t *cnt, int32_t *next, int32_t *next_count,
                                                    int32_t *heavy, int32_t *heavy_count)
{
    const int64_t nf = counters[0];
    for (int64_t f = (int64_t)blockIdx.x * BLOCK + threadIdx.x; f < nf; f += (int64_t)gridDim.x * BLOCK) {
        const int32_t v = front[f];
        const int64_t b = g.off[v], e = g.off[v + 1];
        if (e - b > LIGHT_MAX) {
            heavy[atomicAdd(heavy_count, 1)] = v;
            continue;
        }
        const uint64_t pv = jp_priority(seed, v);
        int32_t c = -1;
        for (int32_t base = 0; c < 0; base += 64) {
            uint64_t used = 0;
            for (int64_t x = b; x < e; ++x) {
                const int32_t u = g.col[x];
                if (u == v || jp_priority(seed, u) < pv) continue;
                const int32_t cu = color[u];
                if (cu >= base && cu < base + 64) used |= 1ull << (cu - base);
            }
            if (used != ~0ull) c = base + __ffsll((unsigned long long)~used) - 1;
        }
        color[v] = c;
        jp_release(g, seed, v, pv, b, e, 1, cnt, next, next_count);
    }
}

// heavy rows: one workgroup per vertex, LDS bitmap of the colours in use
__global__ __launch_bounds__(BLOCK) void k_jp_heavy(Csr g, uint64_t seed, const int32_t *heavy,
                                                    const int32_t *heavy_count, int32_t *color, int32_t *cnt,
                                                    int32_t *next, int32_t *next_count)
{
    __shared__ uint32_t bits[BITMAP_WORDS];
    __shared__ int32_t s_first;
    const int64_t nh = *heavy_count;
    for (int64_t h = blockIdx.x; h < nh; h += gridDim.x) {
        const int32_t v = heavy[h];
        const int64_t b = g.off[v], e = g.off[v + 1];
        const uint64_t pv = jp_priority(seed, v);
        int32_t c = -1;
        for (int32_t base = 0; c < 0; base += BITMAP_WORDS * 32) {
            for (int w = threadIdx.x; w < BITMAP_WORDS; w += BLOCK) bits[w] = 0;
            if (threadIdx.x == 0) s_first = INT32_MAX;
            __syncthreads();
            for (int64_t x = b + threadIdx.x; x < e; x += BLOCK) {
                const int32_t u = g.col[x];
                if (u == v || jp_priority(seed, u) < pv) continue;
                const int32_t cu = color[u] - base;
                if (cu >= 0 && cu < BITMAP_WORDS * 32) atomicOr(&bits[cu >> 5], 1u << (cu & 31));
            }
            __syncthreads();
            for (int w = threadIdx.x; w < BITMAP_WORDS; w += BLOCK)
                if (bits[w] != 0xFFFFFFFFu) atomicMin(&s_first, w * 32 + __ffs(~bits[w]) - 1);
            __syncthreads();
            if (s_first != INT32_MAX) c = base + s_first;
            __syncthreads();
        }
        if (threadIdx.x == 0) color[v] = c;
        jp_release(g, seed, v, pv, b + threadIdx.x, e, BLOCK, cnt, next, next_count);
        __syncthreads();
    }
}

__global__ __launch_bounds__(BLOCK) void k_color_max(const int32_t *color, int64_t n, int32_t *out)
{
    int32_t m = -1;
    for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * BLOCK)
        m = max(m, color[v]);
    atomicMax(out, m);
}

// counters: [0] frontier size, [1] next frontier size, [2] heavy count, [3] colour max
int32_t color_jp(const Csr &g, uint64_t seed, int32_t *color, int32_t *cnt, int32_t *front_a, int32_t *front_b,
                 int32_t *counters, hipStream_t st)
{
    if (g.n == 0) return 0;
    fill<int32_t>(cnt, 0, g.n, st);
    fill<int32_t>(counters, 0, 8, st);
    if (g.nnz > 0) k_jp_count<<<grid_for(g.nnz, ETILE), BLOCK, 0, st>>>(g, seed, cnt);
    unsigned gv = grid_for(g.n, BLOCK * 4);
    if (gv > 65536) gv = 65536;
    k_jp_start<<<gv, BLOCK, 0, st>>>(cnt, g.n, color, front_a, counters);
    int32_t *front = front_a, *next = front_b;
    int32_t *heavy = cnt + g.n; // caller provides cnt with 2n entries
    int64_t colored = 0;
    for (;;) {
        int32_t nf = 0;
        hipMemcpyAsync(&nf, counters, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        hipStreamSynchronize(st);
        if (nf == 0) break;
        colored += nf;
        fill<int32_t>(counters + 1, 0, 2, st);
        unsigned gl = grid_for(nf, BLOCK);
        k_jp_light<<<gl, BLOCK, 0, st>>>(g, seed, front, counters, color, cnt, next, counters + 1, heavy,
                                         counters + 2);
        unsigned gh = nf < 4096 ? (unsigned)nf : 4096u;
        k_jp_heavy<<<gh, BLOCK, 0, st>>>(g, seed, heavy, counters + 2, color, cnt, next, counters + 1);
        // next frontier becomes the current one
        hipMemcpyAsync(counters, counters + 1, sizeof(int32_t), hipMemcpyDeviceToDevice, st);
        int32_t *t = front;
        front = next;
        next = t;
    }
    (void)colored;
    fill<int32_t>(counters + 3, -1, 1, st);
    k_color_max<<<gv, BLOCK, 0, st>>>(color, g.n, counters + 3);
    int32_t mx = -1;
    hipMemcpyAsync(&mx, counters + 3, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    return mx + 1;
}

} // namespace lv
