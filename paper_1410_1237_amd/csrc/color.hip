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
// frontier vertex with a row of up to 256 entries (64-colour register windows),
// a 256-thread workgroup one with up to 4096 entries and a 1024-thread
// workgroup a longer one (LDS bitmap of 4096 colours per window), so every
// row is read a bounded number of times.  Rounds are launched in batches without host synchronisation: the
// frontier sizes live in a small device ring indexed by round; round r reads
// slot r, counts the next frontier into slot r+1 and clears slot r+2 for the
// round after.
#include "lv.h"

namespace lv {

constexpr int JP_WINDOW_WORDS = 64; // 64 x 64 = 4096 colours per window
constexpr unsigned JP_GRID = 512;        // light: 2048 waves per round, grid-stride over the frontier
constexpr unsigned JP_MEDIUM_GRID = 512; // medium: one vertex per 256-thread block, grid-stride
constexpr unsigned JP_HEAVY_GRID = 128;  // heavy: one vertex per 1024-thread block, grid-stride
constexpr int64_t JP_RING = 4; // frontier sizes by round: slots 3 (r % JP_RING) + (light, medium, heavy)

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
// lists are split by row length into light, medium and heavy.
constexpr int64_t JP_MEDIUM = 256;  // rows above: a 256-thread workgroup
constexpr int64_t JP_HEAVY = 4096;  // rows above: a 1024-thread workgroup

struct JpLists {
    int32_t *list[3]; // light, medium, heavy
};

__device__ __forceinline__ void jp_push(const Csr &g, int32_t u, const JpLists &out, int32_t *counts)
{
    const int64_t d = g.off[u + 1] - g.off[u];
    const int k = d > JP_HEAVY ? 2 : (d > JP_MEDIUM ? 1 : 0);
    out.list[k][atomicAdd(&counts[k], 1)] = u;
}

__global__ __launch_bounds__(BLOCK) void k_jp_start(Csr g, const int32_t *cnt, int32_t *color, JpLists out,
                                                    int32_t *ring)
{
    for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < g.n; v += (int64_t)gridDim.x * BLOCK) {
        const int64_t b = g.off[v], e = g.off[v + 1];
        const bool alone = (e == b) || (e - b == 1 && g.col[b] == v);
        color[v] = alone ? 0 : -1;
        if (!alone && cnt[v] == 0) jp_push(g, (int32_t)v, out, ring);
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

// light rows: one wavefront per frontier vertex, colours in 64-colour register
// windows OR-reduced across the wave; waves of a block are independent
__global__ __launch_bounds__(BLOCK) void k_jp_light(Csr g, uint64_t seed, const int32_t *in, int32_t *ring, int64_t r,
                                                    JpLists out, int32_t *color, int32_t *cnt)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (BLOCK / 64);
    int32_t *cur = ring + 3 * (r % JP_RING);
    int32_t *next = ring + 3 * ((r + 1) % JP_RING);
    const int64_t nf = cur[0];
    if (blockIdx.x == 0 && threadIdx.x < 3) ring[3 * ((r + 2) % JP_RING) + threadIdx.x] = 0;
    for (int64_t f = wave; f < nf; f += nwaves) {
        const int32_t v = in[f];
        const int64_t b = g.off[v], e = g.off[v + 1];
        const uint64_t pv = jp_priority(seed, v);
        int32_t c = -1;
        for (int32_t base = 0; c < 0; base += 64) {
            unsigned long long used = 0;
            for (int64_t x = b + lane; x < e; x += 64) {
                const int32_t u = g.col[x];
                if (u == v || jp_priority(seed, u) < pv) continue;
                const int32_t cu = color[u] - base;
                if (cu >= 0 && cu < 64) used |= 1ull << cu;
            }
            used = wave_or(used);
            if (used != ~0ull) c = base + __ffsll(~used) - 1;
        }
        if (lane == 0) color[v] = c;
        for (int64_t x = b + lane; x < e; x += 64) {
            const int32_t u = g.col[x];
            if (u != v && jp_priority(seed, u) < pv)
                if (atomicSub(&cnt[u], 1) == 1) jp_push(g, u, out, next);
        }
    }
}

// medium and heavy rows: one NT-thread workgroup per frontier vertex
template <int NT, int K>
__global__ __launch_bounds__(NT) void k_jp_block(Csr g, uint64_t seed, const int32_t *in, int32_t *ring, int64_t r,
                                                 JpLists out, int32_t *color, int32_t *cnt)
{
    __shared__ unsigned long long bm[JP_WINDOW_WORDS];
    __shared__ int32_t s_c;
    int32_t *cur = ring + 3 * (r % JP_RING);
    int32_t *next = ring + 3 * ((r + 1) % JP_RING);
    const int64_t nf = cur[K];
    for (int64_t f = blockIdx.x; f < nf; f += gridDim.x) {
        const int32_t v = in[f];
        const int64_t b = g.off[v], e = g.off[v + 1];
        const uint64_t pv = jp_priority(seed, v);
        const int32_t c = jp_mex<NT>(g, seed, v, pv, b, e, color, bm, &s_c);
        if (threadIdx.x == 0) color[v] = c;
        for (int64_t x = b + threadIdx.x; x < e; x += NT) {
            const int32_t u = g.col[x];
            if (u != v && jp_priority(seed, u) < pv)
                if (atomicSub(&cnt[u], 1) == 1) jp_push(g, u, out, next);
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

// ring needs 3 JP_RING + 1 entries (<= 16); cnt needs 5n entries (counts, then
// the medium and heavy frontier lists, two each); front_a / front_b are the
// light lists (n each)
int32_t color_jp(const Csr &g, uint64_t seed, int32_t *color, int32_t *cnt, int32_t *front_a, int32_t *front_b,
                 int32_t *ring, hipStream_t st)
{
    if (g.n == 0) return 0;
    fill<int32_t>(cnt, 0, g.n, st);
    fill<int32_t>(ring, 0, 3 * JP_RING + 1, st);
    if (g.nnz > 0) k_jp_count<<<grid_for(g.nnz, ETILE), BLOCK, 0, st>>>(g, seed, cnt);
    unsigned gv = grid_for(g.n, BLOCK * 4);
    if (gv > 65536) gv = 65536;
    JpLists lists[2] = {{{front_a, cnt + g.n, cnt + 3 * g.n}}, {{front_b, cnt + 2 * g.n, cnt + 4 * g.n}}};
    k_jp_start<<<gv, BLOCK, 0, st>>>(g, cnt, color, lists[0], ring);
    int64_t r = 0;     // next round to launch
    int64_t batch = 4; // rounds launched per host check, doubled up to 256
    for (;;) {
        for (int64_t i = 0; i < batch; ++i, ++r) {
            const JpLists &in = lists[r & 1], &out = lists[(r + 1) & 1];
            k_jp_light<<<JP_GRID, BLOCK, 0, st>>>(g, seed, in.list[0], ring, r, out, color, cnt);
            k_jp_block<BLOCK, 1><<<JP_MEDIUM_GRID, BLOCK, 0, st>>>(g, seed, in.list[1], ring, r, out, color, cnt);
            k_jp_block<1024, 2><<<JP_HEAVY_GRID, 1024, 0, st>>>(g, seed, in.list[2], ring, r, out, color, cnt);
        }
        int32_t nf[3] = {0, 0, 0};
        hipMemcpyAsync(nf, ring + 3 * (r % JP_RING), 3 * sizeof(int32_t), hipMemcpyDeviceToHost, st);
        hipStreamSynchronize(st);
        if (nf[0] == 0 && nf[1] == 0 && nf[2] == 0) break;
        if (batch < 256) batch *= 2;
    }
    int32_t *mx_slot = ring + 3 * JP_RING;
    fill<int32_t>(mx_slot, -1, 1, st);
    k_color_max<<<gv, BLOCK, 0, st>>>(color, g.n, mx_slot);
    int32_t mx = -1;
    hipMemcpyAsync(&mx, mx_slot, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    return mx + 1;
}

} // namespace lv
