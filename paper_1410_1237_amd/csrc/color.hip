// Distance-1 coloring (Sec. 5.2) by Jones-Plassmann rounds with hashed
// priorities pi(v) = SplitMix64 finalizer((seed << 32) ^ v) (Steele, Lea,
// Flood 2014).  Priorities are a bijection of v, so every vertex has a
// strict rank; a vertex is coloured once all its higher-priority neighbours
// are, with the smallest colour none of them uses.  The result is therefore
// exactly the greedy colouring in descending priority, for any schedule.
//
// Each vertex keeps the count of its uncoloured higher-priority neighbours;
// colouring a vertex decrements its lower-priority neighbours and those
// reaching zero form the next round's frontier.  One wavefront colours one
// frontier vertex (LDS bitmap of the colours its higher-priority neighbours
// use, 4096 colours per window), so every row is read a bounded number of
// times.  Rounds are launched in batches without host synchronisation: the
// frontier sizes live in a small device ring indexed by round; round r reads
// slot r, counts the next frontier into slot r+1 and clears slot r+2 for the
// round after.
#include "lv.h"

namespace lv {

constexpr int JP_WINDOW_WORDS = 64; // 64 x 64 = 4096 colours per window
constexpr unsigned JP_GRID = 8192;  // light blocks (one wave each) per round, grid-stride over the frontier
constexpr unsigned JP_HEAVY_GRID = 512;
constexpr int64_t JP_RING = 6; // frontier sizes by round: slots 2(r % JP_RING) (light) and +1 (heavy)

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
        if (u == v) continue;
        if (jp_priority(seed, u) > jp_priority(seed, v)) atomicAdd(&cnt[v], 1);
    }
}

// vertices without higher-priority neighbours start the frontier; a vertex
// with no neighbour other than itself takes colour 0 at once.  Frontier
// lists are split by row length: light rows go to one wavefront each, heavy
// rows (> JP_HEAVY entries) to a 1024-thread workgroup each.
constexpr int64_t JP_HEAVY = 4096;
constexpr int JP_HEAVY_BLOCK = 1024;

__device__ __forceinline__ void jp_push(const Csr &g, int32_t u, int32_t *light, int32_t *heavy, int32_t *counts)
{
    if (g.off[u + 1] - g.off[u] > JP_HEAVY) heavy[atomicAdd(&counts[1], 1)] = u;
    else light[atomicAdd(&counts[0], 1)] = u;
}

__global__ __launch_bounds__(BLOCK) void k_jp_start(Csr g, const int32_t *cnt, int32_t *color, int32_t *light,
                                                    int32_t *heavy, int32_t *ring)
{
    for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < g.n; v += (int64_t)gridDim.x * BLOCK) {
        const int64_t b = g.off[v], e = g.off[v + 1];
        const bool alone = (e == b) || (e - b == 1 && g.col[b] == v);
        color[v] = alone ? 0 : -1;
        if (!alone && cnt[v] == 0) jp_push(g, (int32_t)v, light, heavy, ring);
    }
}

// smallest colour not used by the higher-priority neighbours of v, computed
// by the NT threads of the block with an LDS bitmap per window of 4096 colours
template <int NT>
__device__ __forceinline__ int32_t jp_mex(const Csr &g, uint64_t seed, int32_t v, uint64_t pv, int64_t b, int64_t e,
                                          const int32_t *color, unsigned long long *bm, int32_t *s_c)
{
    int32_t c = -1;
    for (int32_t base = 0; c < 0; base += JP_WINDOW_WORDS * 64) {
        if (threadIdx.x < JP_WINDOW_WORDS) bm[threadIdx.x] = 0;
        __syncthreads();
        for (int64_t x = b + threadIdx.x; x < e; x += NT) {
            const int32_t u = g.col[x];
            if (u == v || jp_priority(seed, u) < pv) continue;
            const int32_t cu = color[u] - base;
            if (cu >= 0 && cu < JP_WINDOW_WORDS * 64) atomicOr(&bm[cu >> 6], 1ull << (cu & 63));
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            const unsigned long long word = bm[threadIdx.x];
            const unsigned long long open = __ballot(word != ~0ull);
            if (threadIdx.x == 0) {
                int32_t r = -1;
                if (open) {
                    const int l = __ffsll(open) - 1;
                    r = base + l * 64 + __ffsll(~bm[l]) - 1;
                }
                *s_c = r;
            }
        }
        __syncthreads();
        c = *s_c;
        __syncthreads();
    }
    return c;
}

// one round over the light and heavy frontier lists of slot r
template <int NT, bool HEAVY>
__global__ __launch_bounds__(NT) void k_jp_round(Csr g, uint64_t seed, const int32_t *in_light, const int32_t *in_heavy,
                                                 int32_t *ring, int64_t r, int32_t *out_light, int32_t *out_heavy,
                                                 int32_t *color, int32_t *cnt)
{
    __shared__ unsigned long long bm[JP_WINDOW_WORDS];
    __shared__ int32_t s_c;
    int32_t *cur = ring + 2 * (r % JP_RING);
    int32_t *next = ring + 2 * ((r + 1) % JP_RING);
    const int64_t nf = HEAVY ? cur[1] : cur[0];
    const int32_t *front = HEAVY ? in_heavy : in_light;
    if (!HEAVY && blockIdx.x == 0 && threadIdx.x < 2) ring[2 * ((r + 2) % JP_RING) + threadIdx.x] = 0;
    for (int64_t f = blockIdx.x; f < nf; f += gridDim.x) {
        const int32_t v = front[f];
        const int64_t b = g.off[v], e = g.off[v + 1];
        const uint64_t pv = jp_priority(seed, v);
        const int32_t c = jp_mex<NT>(g, seed, v, pv, b, e, color, bm, &s_c);
        if (threadIdx.x == 0) color[v] = c;
        for (int64_t x = b + threadIdx.x; x < e; x += NT) {
            const int32_t u = g.col[x];
            if (u != v && jp_priority(seed, u) < pv)
                if (atomicSub(&cnt[u], 1) == 1) jp_push(g, u, out_light, out_heavy, next);
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_color_max(const int32_t *color, int64_t n, int32_t *out)
{
    int32_t m = -1;
    for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * BLOCK)
        m = max(m, color[v]);
    atomicMax(out, m);
}

// ring needs 2 JP_RING + 1 entries (<= 16); cnt needs 3n entries (counts, then
// the two heavy frontier lists); front_a / front_b are the light lists (n each)
int32_t color_jp(const Csr &g, uint64_t seed, int32_t *color, int32_t *cnt, int32_t *front_a, int32_t *front_b,
                 int32_t *ring, hipStream_t st)
{
    if (g.n == 0) return 0;
    fill<int32_t>(cnt, 0, g.n, st);
    fill<int32_t>(ring, 0, 2 * JP_RING + 1, st);
    if (g.nnz > 0) k_jp_count<<<grid_for(g.nnz, ETILE), BLOCK, 0, st>>>(g, seed, cnt);
    unsigned gv = grid_for(g.n, BLOCK * 4);
    if (gv > 65536) gv = 65536;
    int32_t *heavy[2] = {cnt + g.n, cnt + 2 * g.n};
    int32_t *light[2] = {front_a, front_b};
    k_jp_start<<<gv, BLOCK, 0, st>>>(g, cnt, color, light[0], heavy[0], ring);
    int64_t r = 0;     // next round to launch
    int64_t batch = 4; // rounds launched per host check, doubled up to 256
    for (;;) {
        for (int64_t i = 0; i < batch; ++i, ++r) {
            const int a = r & 1, b = (r + 1) & 1;
            k_jp_round<64, false><<<JP_GRID, 64, 0, st>>>(g, seed, light[a], heavy[a], ring, r, light[b], heavy[b],
                                                          color, cnt);
            k_jp_round<JP_HEAVY_BLOCK, true><<<JP_HEAVY_GRID, JP_HEAVY_BLOCK, 0, st>>>(
                g, seed, light[a], heavy[a], ring, r, light[b], heavy[b], color, cnt);
        }
        int32_t nf[2] = {0, 0};
        hipMemcpyAsync(nf, ring + 2 * (r % JP_RING), 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st);
        hipStreamSynchronize(st);
        if (nf[0] == 0 && nf[1] == 0) break;
        if (batch < 256) batch *= 2;
    }
    int32_t *mx_slot = ring + 2 * JP_RING;
    fill<int32_t>(mx_slot, -1, 1, st);
    k_color_max<<<gv, BLOCK, 0, st>>>(color, g.n, mx_slot);
    int32_t mx = -1;
    hipMemcpyAsync(&mx, mx_slot, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    return mx + 1;
}

} // namespace lv
