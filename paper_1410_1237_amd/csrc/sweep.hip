// The synchronous local-moving sweep (Alg. 1 inner loop, Eq. 1, 4, 5 and the
// minimum-label heuristics of Sec. 5.1) as degree-binned gfx950 kernels.
//
// Every vertex of a launch reads only the state of the previous iteration
// (or colour class): comm_prev, a (community degrees) and size.  A group of
// LPV lanes gathers the vertex's row, sums the edge weight per neighbouring
// community e_{i->c} in an open-addressed hash table (LDS for rows up to
// 2048 entries, a per-vertex HBM table for hubs), then evaluates the exact
// integer gain G(c) = 2m*e_{i->c} - k_i*a_c for every distinct community and
// reduces the lexicographic maximum of (G, -c) with wave shuffles.  The
// vertex moves iff G(c*) > G_stay = 2m*e_{i->A\{i}} - k_i*(a_A - k_i) and the
// singlet rule does not veto (A and c* both single-vertex and c* > A).
//
// Integer sums make every result independent of the order of atomics, so
// the output is deterministic for any launch shape.
#include "lv.h"

#include <type_traits>

namespace lv {

template <typename T> __device__ __forceinline__ T shfl_xor_t(T v, int mask, int width)
{
    constexpr int W = sizeof(T) / 4;
    union {
        T t;
        int w[W];
    } u;
    u.t = v;
#pragma unroll
    for (int k = 0; k < W; ++k) u.w[k] = __shfl_xor(u.w[k], mask, width);
    return u.t;
}

template <typename GT> struct Best {
    GT g;      // gain of the best candidate
    int32_t c; // its community (-1: none)
    int64_t e; // its e_{i->c}
};

template <typename GT> __device__ __forceinline__ bool better(const Best<GT> &x, const Best<GT> &y)
{
    if (y.c < 0) return x.c >= 0;
    if (x.c < 0) return false;
    return x.g > y.g || (x.g == y.g && x.c < y.c);
}

__device__ __forceinline__ uint32_t slot_hash(int32_t c, int shift)
{
    return ((uint32_t)c * 0x9E3779B1u) >> (32 - shift);
}

__device__ __forceinline__ int64_t two_m_of(const SweepArgs &a, int32_t v)
{
    return a.gid ? a.two_m_g[a.gid[v]] : a.two_m;
}

__device__ __forceinline__ bool sweeping(const SweepArgs &a, int32_t v)
{
    return !a.gid || a.active_g[a.gid[v]] != 0;
}

// per-graph stats of a batched sweep: one record per vertex group, runs of
// equal graph ids folded by one thread (the vertices of a block are sorted by
// id, so their graphs form few runs) before the global atomics
template <int VPB>
__device__ __forceinline__ void flush_graph_stats(const SweepArgs &a, int grp, bool leader, int32_t g,
                                                  const int64_t v[5])
{
    __shared__ int64_t rec[VPB][5];
    __shared__ int32_t rg[VPB];
    if (leader) {
        rg[grp] = g;
        for (int k = 0; k < 5; ++k) rec[grp][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t cur = -1;
        int64_t acc[5] = {0, 0, 0, 0, 0};
        for (int q = 0; q <= VPB; ++q) {
            const int32_t gq = q < VPB ? rg[q] : -2;
            if (gq != cur) {
                if (cur >= 0)
                    for (int k = 0; k < 5; ++k)
                        if (acc[k]) atomicAdd((unsigned long long *)&a.gstats[8 * (int64_t)cur + k], (unsigned long long)acc[k]);
                cur = gq;
                for (int k = 0; k < 5; ++k) acc[k] = 0;
            }
            if (q < VPB && gq >= 0)
                for (int k = 0; k < 5; ++k) acc[k] += rec[q][k];
        }
    }
}

// One block-tile of a degree bin: VPB = BLOCK / LPV vertices, LPV lanes each,
// hash tables of 2^shift slots per vertex in LDS.
template <int LPV, int WK, typename GT>
__device__ __forceinline__ void sweep_tile(const SweepArgs &a, const BinRange &br, int64_t tile, int shift,
                                           unsigned char *smem, unsigned long long *bstat)
{
    typedef typename std::conditional<WK == W_UNIT, uint32_t, unsigned long long>::type VT;
    constexpr int VPB = BLOCK / LPV;
    const int grp = threadIdx.x / LPV, lane = threadIdx.x % LPV;
    const int64_t vidx = tile * VPB + grp;
    const int32_t i = vidx < br.count ? br.verts[vidx] : 0;
    const bool valid = vidx < br.count && sweeping(a, i);
    const int64_t two_m = valid ? two_m_of(a, i) : 0;

    const int64_t S = (int64_t)1 << shift;
    int32_t *tkey = (int32_t *)smem + grp * S;
    VT *tval = (VT *)(smem + (size_t)VPB * S * sizeof(int32_t)) + grp * S;
    for (int64_t s = lane; s < S; s += LPV) {
        tkey[s] = -1;
        tval[s] = 0;
    }
    if (threadIdx.x < 5) bstat[threadIdx.x] = 0;
    __syncthreads();

    // gather: e_{i->c} per neighbouring community (Eq. 1), self-loop apart
    int64_t beg = 0, end = 0, wself = 0;
    int32_t A = 0;
    if (valid) {
        beg = a.g.off[i];
        end = a.g.off[i + 1];
        A = a.comm_prev[i];
    }
    for (int64_t e = beg + lane; e < end; e += LPV) {
        const int32_t j = a.g.col[e];
        const int64_t w = WLoad<WK>::at(a.g.w, e);
        if (j == i) {
            wself += w;
            continue;
        }
        const int32_t c = a.comm_prev[j];
        uint32_t h = slot_hash(c, shift);
        for (;;) {
            int32_t cur = tkey[h];
            if (cur == c) {
                atomicAdd(&tval[h], (VT)w);
                break;
            }
            if (cur == -1) {
                cur = atomicCAS(&tkey[h], -1, c);
                if (cur == -1 || cur == c) {
                    atomicAdd(&tval[h], (VT)w);
                    break;
                }
            }
            h = (h + 1) & (uint32_t)(S - 1);
        }
    }
    __syncthreads();

    // gains over the distinct communities (Eq. 4 scaled by 2m^2), best by (G, -c)
    const int64_t ki = valid ? a.k[i] : 0;
    Best<GT> best{0, -1, 0};
    int64_t eA = 0, distinct = 0;
    for (int64_t s = lane; s < S; s += LPV) {
        const int32_t c = tkey[s];
        if (c < 0) continue;
        const int64_t e = (int64_t)tval[s];
        ++distinct;
        if (c == A) {
            eA = e;
            continue;
        }
        Best<GT> cand{(GT)two_m * (GT)e - (GT)ki * (GT)a.a[c], c, e};
        if (better(cand, best)) best = cand;
    }

    // reduce over the LPV lanes of the vertex
    constexpr int WRED = LPV < 64 ? LPV : 64;
#pragma unroll
    for (int m = 1; m < WRED; m <<= 1) {
        Best<GT> o;
        o.g = shfl_xor_t(best.g, m, WRED);
        o.c = shfl_xor_t(best.c, m, WRED);
        o.e = shfl_xor_t(best.e, m, WRED);
        if (better(o, best)) best = o;
        eA += shfl_xor_t(eA, m, WRED);
        wself += shfl_xor_t(wself, m, WRED);
        distinct += shfl_xor_t(distinct, m, WRED);
    }
    if (LPV > 64) {
        __shared__ Best<GT> sb[BLOCK / 64];
        __shared__ int64_t se[BLOCK / 64][3];
        const int wid = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            sb[wid] = best;
            se[wid][0] = eA;
            se[wid][1] = wself;
            se[wid][2] = distinct;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < BLOCK / 64; ++w) {
                if (better(sb[w], best)) best = sb[w];
                eA += se[w][0];
                wself += se[w][1];
                distinct += se[w][2];
            }
        }
    }

    // decision (Alg. 1: move iff the best gain beats staying; Sec. 5.1 singlet rule)
    int64_t vs[5] = {0, 0, 0, 0, 0};
    if (lane == 0 && valid) {
        const GT stay = (GT)two_m * (GT)eA - (GT)ki * (GT)(a.a[A] - ki);
        bool move = best.c >= 0 && best.g > stay;
        if (move && a.singlet && a.size[A] == 1 && a.size[best.c] == 1 && best.c > A) move = false;
        a.comm_next[i] = move ? best.c : A;
        vs[0] = move ? 1 : 0;
        vs[1] = eA + wself;
        vs[2] = move ? 2 * (best.e - eA) : 0;
        vs[3] = distinct;
        vs[4] = end - beg;
    }
    if (a.gid) {
        flush_graph_stats<VPB>(a, grp, lane == 0, valid ? a.gid[i] : -1, vs);
        return;
    }
    if (lane == 0 && valid) {
        if (vs[0]) atomicAdd(&bstat[0], 1ull);
        if (vs[2]) atomicAdd(&bstat[2], (unsigned long long)vs[2]);
        atomicAdd(&bstat[1], (unsigned long long)vs[1]);
        atomicAdd(&bstat[3], (unsigned long long)vs[3]);
        atomicAdd(&bstat[4], (unsigned long long)vs[4]);
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        const unsigned long long v = bstat[threadIdx.x];
        if (v) atomicAdd((unsigned long long *)&br.stats->moves + threadIdx.x, v);
    }
}

// hubs: rows longer than 2048 entries -----------------------------------------
// (1) insert: each block pre-aggregates a 2048-entry chunk of one hub row in an
// LDS table, then adds its distinct communities to the hub's HBM table;
// (2) scan: each block reads a 4096-slot slice of one hub table, leaves it
// clean and keeps the slice's best (G, -c); (3) decide: one thread per hub
// reduces its slices and applies the same rule as the other bins.
constexpr int HUB_LDS = 2 * HUB_CHUNK;

__device__ __forceinline__ int64_t last_leq(const int64_t *arr, int64_t lo, int64_t hi, int64_t x)
{
    // largest p in [lo, hi) with arr[p] <= x (arr non-decreasing, arr[lo] <= x)
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (arr[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// Merges the occupied slots of a block's LDS table (HUB_LDS slots) into an
// HBM table of S slots.  Each thread holds its PER slots in registers and
// issues their compare-and-swaps together, so up to PER device-coherent
// atomics per thread are in flight instead of one.
constexpr int FLUSH_PER = HUB_LDS / BLOCK;

__device__ __forceinline__ void flush_to_hbm(const int32_t *tkey, const unsigned long long *tval, int32_t *gkey,
                                             unsigned long long *gval, int64_t S, int gshift)
{
    int32_t kc[FLUSH_PER];
    unsigned long long kv[FLUSH_PER];
    uint32_t kq[FLUSH_PER];
    uint32_t pend = 0;
#pragma unroll
    for (int j = 0; j < FLUSH_PER; ++j) {
        const int s = threadIdx.x + j * BLOCK;
        kc[j] = tkey[s];
        kv[j] = tval[s];
        kq[j] = kc[j] >= 0 ? slot_hash(kc[j], gshift) : 0;
        if (kc[j] >= 0) pend |= 1u << j;
    }
    while (pend) {
        int32_t old[FLUSH_PER];
#pragma unroll
        for (int j = 0; j < FLUSH_PER; ++j)
            if ((pend >> j) & 1) old[j] = atomicCAS(&gkey[kq[j]], -1, kc[j]);
#pragma unroll
        for (int j = 0; j < FLUSH_PER; ++j) {
            if (!((pend >> j) & 1)) continue;
            if (old[j] == -1 || old[j] == kc[j]) {
                atomicAdd(&gval[kq[j]], kv[j]);
                pend &= ~(1u << j);
            } else {
                kq[j] = (kq[j] + 1) & (uint32_t)(S - 1);
            }
        }
    }
}

// Reads (and clears) HBM table slots [base, base + count) with SCAN_PER
// independent loads in flight per thread; calls f(community, weight) for
// each occupied slot.
constexpr int SCAN_PER = 16;

template <class F>
__device__ __forceinline__ void scan_hbm(int32_t *gkey, unsigned long long *gval, int64_t count, F f)
{
    for (int64_t base = 0; base < count; base += (int64_t)BLOCK * SCAN_PER) {
        int32_t c[SCAN_PER];
#pragma unroll
        for (int j = 0; j < SCAN_PER; ++j) {
            const int64_t s = base + threadIdx.x + (int64_t)j * BLOCK;
            c[j] = s < count ? __hip_atomic_load(&gkey[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : -1;
        }
        unsigned long long w[SCAN_PER];
#pragma unroll
        for (int j = 0; j < SCAN_PER; ++j) {
            const int64_t s = base + threadIdx.x + (int64_t)j * BLOCK;
            w[j] = c[j] >= 0 ? __hip_atomic_load(&gval[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
        }
#pragma unroll
        for (int j = 0; j < SCAN_PER; ++j) {
            if (c[j] < 0) continue;
            const int64_t s = base + threadIdx.x + (int64_t)j * BLOCK;
            gkey[s] = -1; // leave the table clean for the next sweep
            gval[s] = 0;
            f(c[j], (int64_t)w[j]);
        }
    }
}

template <int WK>
__device__ __forceinline__ void hub_insert_tile(const SweepArgs &a, const HubArgs &h, int64_t tile, unsigned char *smem,
                                                int64_t *red)
{
    int32_t *tkey = (int32_t *)smem;
    unsigned long long *tval = (unsigned long long *)(smem + HUB_LDS * sizeof(int32_t));
    const int64_t target = h.chunk0 + tile;
    const int64_t p = last_leq(h.cpre, h.s, h.e, target);
    const int32_t v = h.verts[p];
    if (!sweeping(a, v)) return; // uniform over the block
    const int64_t rb = a.g.off[v], re = a.g.off[v + 1];
    const int64_t beg = rb + (target - h.cpre[p]) * HUB_CHUNK;
    const int64_t end = min(re, beg + HUB_CHUNK);
    for (int s = threadIdx.x; s < HUB_LDS; s += BLOCK) {
        tkey[s] = -1;
        tval[s] = 0;
    }
    __syncthreads();
    constexpr int shift = 12; // log2(HUB_LDS)
    int64_t wself = 0;
    for (int64_t e = beg + threadIdx.x; e < end; e += BLOCK) {
        const int32_t j = a.g.col[e];
        const int64_t w = WLoad<WK>::at(a.g.w, e);
        if (j == v) {
            wself += w;
            continue;
        }
        const int32_t c = a.comm_prev[j];
        uint32_t q = slot_hash(c, shift);
        for (;;) {
            int32_t cur = tkey[q];
            if (cur == c) {
                atomicAdd(&tval[q], (unsigned long long)w);
                break;
            }
            if (cur == -1) {
                cur = atomicCAS(&tkey[q], -1, c);
                if (cur == -1 || cur == c) {
                    atomicAdd(&tval[q], (unsigned long long)w);
                    break;
                }
            }
            q = (q + 1) & (HUB_LDS - 1);
        }
    }
    __syncthreads();
    const int64_t t0 = h.hoff[p], S = h.hoff[p + 1] - t0;
    const int gshift = __ffsll((unsigned long long)S) - 1;
    int32_t *gkey = h.hkey + t0;
    unsigned long long *gval = (unsigned long long *)h.hval + t0;
    flush_to_hbm(tkey, tval, gkey, gval, S, gshift);
    // self-loop weight and entry count of the chunk
    int64_t x = wself;
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) x += shfl_xor_t(x, m, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int w = 0; w < BLOCK / 64; ++w) t += red[w];
        int64_t *aux = h.aux + 8 * (t0 / HUB_SLICE);
        if (t) atomicAdd((unsigned long long *)&aux[0], (unsigned long long)t);
        atomicAdd((unsigned long long *)&aux[1], (unsigned long long)(end - beg));
    }
}

// mid hubs (bin 9): one workgroup per vertex; the row is pre-aggregated per
// 2048-entry chunk in LDS, merged into the vertex's HBM table, and the same
// workgroup scans (and clears) the table and decides.
template <int WK, typename GT>
__device__ __forceinline__ void mid_hub_tile(const SweepArgs &a, const BinRange &br, const FusedBins &f,
                                             int64_t tile, unsigned char *smem, unsigned long long *bstat)
{
    __shared__ Best<GT> sb[BLOCK / 64];
    __shared__ int64_t se[BLOCK / 64][3];
    int32_t *tkey = (int32_t *)smem;
    unsigned long long *tval = (unsigned long long *)(smem + HUB_LDS * sizeof(int32_t));
    const int32_t i = br.verts[tile];
    if (!sweeping(a, i)) return; // uniform over the block
    const int64_t two_m = two_m_of(a, i);
    const int64_t rb = a.g.off[i], re = a.g.off[i + 1];
    const int64_t t0 = f.hoff9[tile], S = f.hoff9[tile + 1] - t0;
    const int gshift = __ffsll((unsigned long long)S) - 1;
    int32_t *gkey = f.hkey + t0;
    unsigned long long *gval = (unsigned long long *)f.hval + t0;
    (void)bstat;
    int64_t wself = 0;
    for (int64_t cb = rb; cb < re; cb += HUB_CHUNK) {
        const int64_t ce = min(re, cb + HUB_CHUNK);
        for (int s = threadIdx.x; s < HUB_LDS; s += BLOCK) {
            tkey[s] = -1;
            tval[s] = 0;
        }
        __syncthreads();
        for (int64_t e = cb + threadIdx.x; e < ce; e += BLOCK) {
            const int32_t j = a.g.col[e];
            const int64_t w = WLoad<WK>::at(a.g.w, e);
            if (j == i) {
                wself += w;
                continue;
            }
            const int32_t c = a.comm_prev[j];
            uint32_t q = slot_hash(c, 12);
            for (;;) {
                int32_t cur = tkey[q];
                if (cur == c) {
                    atomicAdd(&tval[q], (unsigned long long)w);
                    break;
                }
                if (cur == -1) {
                    cur = atomicCAS(&tkey[q], -1, c);
                    if (cur == -1 || cur == c) {
                        atomicAdd(&tval[q], (unsigned long long)w);
                        break;
                    }
                }
                q = (q + 1) & (HUB_LDS - 1);
            }
        }
        __syncthreads();
        flush_to_hbm(tkey, tval, gkey, gval, S, gshift);
        __threadfence();
        __syncthreads();
    }
    const int32_t A = a.comm_prev[i];
    const int64_t ki = a.k[i];
    Best<GT> best{0, -1, 0};
    int64_t eA = 0, distinct = 0;
    scan_hbm(gkey, gval, S, [&](int32_t c, int64_t e) {
        ++distinct;
        if (c == A) {
            eA = e;
            return;
        }
        Best<GT> cand{(GT)two_m * (GT)e - (GT)ki * (GT)a.a[c], c, e};
        if (better(cand, best)) best = cand;
    });
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        Best<GT> o;
        o.g = shfl_xor_t(best.g, m, 64);
        o.c = shfl_xor_t(best.c, m, 64);
        o.e = shfl_xor_t(best.e, m, 64);
        if (better(o, best)) best = o;
        eA += shfl_xor_t(eA, m, 64);
        wself += shfl_xor_t(wself, m, 64);
        distinct += shfl_xor_t(distinct, m, 64);
    }
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sb[wid] = best;
        se[wid][0] = eA;
        se[wid][1] = wself;
        se[wid][2] = distinct;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < BLOCK / 64; ++w) {
            if (better(sb[w], best)) best = sb[w];
            eA += se[w][0];
            wself += se[w][1];
            distinct += se[w][2];
        }
        const GT stay = (GT)two_m * (GT)eA - (GT)ki * (GT)(a.a[A] - ki);
        bool move = best.c >= 0 && best.g > stay;
        if (move && a.singlet && a.size[A] == 1 && a.size[best.c] == 1 && best.c > A) move = false;
        a.comm_next[i] = move ? best.c : A;
        unsigned long long *st =
            a.gid ? (unsigned long long *)&a.gstats[8 * (int64_t)a.gid[i]] : (unsigned long long *)&br.stats->moves;
        if (move) {
            atomicAdd(&st[0], 1ull);
            atomicAdd(&st[2], (unsigned long long)(2 * (best.e - eA)));
        }
        atomicAdd(&st[1], (unsigned long long)(eA + wself));
        atomicAdd(&st[3], (unsigned long long)distinct);
        atomicAdd(&st[4], (unsigned long long)(re - rb));
    }
}

// Fused launches: blocks are assigned to bins by block ranges.
//  small: bins 1..5 (4..64 lanes per vertex, 512 LDS slots per block)
//  large: bins 6..8 (64 or 256 lanes per vertex, up to 4096 slots) and the hub chunk inserts
template <int WK, typename GT>
__global__ __launch_bounds__(BLOCK) void k_sweep_small(SweepArgs a, FusedBins f)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned long long bstat[5];
    const int64_t blk = blockIdx.x;
    int b = 1;
    while (b < 5 && blk >= f.bins[b + 1].block0) ++b;
    const int64_t tile = blk - f.bins[b].block0;
    switch (b) {
    case 1: sweep_tile<4, WK, GT>(a, f.bins[1], tile, 3, smem, bstat); break;
    case 2: sweep_tile<8, WK, GT>(a, f.bins[2], tile, 4, smem, bstat); break;
    case 3: sweep_tile<16, WK, GT>(a, f.bins[3], tile, 5, smem, bstat); break;
    case 4: sweep_tile<32, WK, GT>(a, f.bins[4], tile, 6, smem, bstat); break;
    default: sweep_tile<64, WK, GT>(a, f.bins[5], tile, 7, smem, bstat); break;
    }
}

template <int WK, typename GT>
__global__ __launch_bounds__(BLOCK) void k_sweep_large(SweepArgs a, FusedBins f, HubArgs h)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned long long bstat[5];
    __shared__ int64_t red[BLOCK / 64];
    const int64_t blk = blockIdx.x;
    if (blk >= f.hub_block0) {
        hub_insert_tile<WK>(a, h, blk - f.hub_block0, smem, red);
        return;
    }
    int b = 6;
    while (b < 9 && blk >= f.bins[b + 1].block0) ++b;
    const int64_t tile = blk - f.bins[b].block0;
    switch (b) {
    case 6: sweep_tile<64, WK, GT>(a, f.bins[6], tile, 9, smem, bstat); break;
    case 7: sweep_tile<256, WK, GT>(a, f.bins[7], tile, 11, smem, bstat); break;
    case 8: sweep_tile<256, WK, GT>(a, f.bins[8], tile, 12, smem, bstat); break;
    default: mid_hub_tile<WK, GT>(a, f.bins[9], f, tile, smem, bstat); break;
    }
}

// decision of giant hub p from its slice records (called by the last slice block)
template <typename GT> __device__ void hub_decide_one(const SweepArgs &a, const HubArgs &h, int64_t p)
{
    const int32_t v = h.verts[p];
    const int64_t first = h.hoff[p] / HUB_SLICE, last = h.hoff[p + 1] / HUB_SLICE;
    Best<GT> best{0, -1, 0};
    for (int64_t q = first; q < last; ++q) {
        int64_t *rec = h.part + 4 * q;
        const uint64_t lo = (uint64_t)__hip_atomic_load(&rec[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int64_t hi = __hip_atomic_load(&rec[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const i128 g = (i128)(((u128)(uint64_t)hi << 64) | (u128)lo);
        Best<GT> cand{(GT)g, (int32_t)__hip_atomic_load(&rec[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                      __hip_atomic_load(&rec[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)};
        if (better(cand, best)) best = cand;
    }
    int64_t *aux = h.aux + 8 * first;
    const int64_t wself = __hip_atomic_load(&aux[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t entries = __hip_atomic_load(&aux[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t eA = __hip_atomic_load(&aux[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t distinct = __hip_atomic_load(&aux[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int t = 0; t < 5; ++t) __hip_atomic_store(&aux[t], (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t A = a.comm_prev[v];
    const int64_t kv = a.k[v];
    const GT stay = (GT)two_m_of(a, v) * (GT)eA - (GT)kv * (GT)(a.a[A] - kv);
    bool move = best.c >= 0 && best.g > stay;
    if (move && a.singlet && a.size[A] == 1 && a.size[best.c] == 1 && best.c > A) move = false;
    a.comm_next[v] = move ? best.c : A;
    unsigned long long *st =
        a.gid ? (unsigned long long *)&a.gstats[8 * (int64_t)a.gid[v]] : (unsigned long long *)&a.stats->moves;
    if (move) {
        atomicAdd(&st[0], 1ull);
        atomicAdd(&st[2], (unsigned long long)(2 * (best.e - eA)));
    }
    atomicAdd(&st[1], (unsigned long long)(eA + wself));
    atomicAdd(&st[3], (unsigned long long)distinct);
    atomicAdd(&st[4], (unsigned long long)entries);
}

// scan of one 4096-slot slice of a giant-hub table; the last slice block of a
// hub (counted in aux[4]) makes the hub's decision
template <typename GT>
__global__ __launch_bounds__(BLOCK) void k_hub_scan(SweepArgs a, HubArgs h)
{
    __shared__ Best<GT> sb[BLOCK / 64];
    __shared__ int64_t se[BLOCK / 64][2];
    const int64_t slice = h.slice0 + blockIdx.x;
    const int64_t p = last_leq(h.hoff, h.s, h.e, slice * HUB_SLICE);
    const int32_t v = h.verts[p];
    if (!sweeping(a, v)) return; // uniform over the block
    const int64_t two_m = two_m_of(a, v);
    const int32_t A = a.comm_prev[v];
    const int64_t kv = a.k[v];
    Best<GT> best{0, -1, 0};
    int64_t eA = 0, distinct = 0;
    const int64_t base = slice * HUB_SLICE;
    scan_hbm(h.hkey + base, (unsigned long long *)h.hval + base, HUB_SLICE, [&](int32_t c, int64_t e) {
        ++distinct;
        if (c == A) {
            eA += e;
            return;
        }
        Best<GT> cand{(GT)two_m * (GT)e - (GT)kv * (GT)a.a[c], c, e};
        if (better(cand, best)) best = cand;
    });
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        Best<GT> o;
        o.g = shfl_xor_t(best.g, m, 64);
        o.c = shfl_xor_t(best.c, m, 64);
        o.e = shfl_xor_t(best.e, m, 64);
        if (better(o, best)) best = o;
        eA += shfl_xor_t(eA, m, 64);
        distinct += shfl_xor_t(distinct, m, 64);
    }
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sb[wid] = best;
        se[wid][0] = eA;
        se[wid][1] = distinct;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < BLOCK / 64; ++w) {
            if (better(sb[w], best)) best = sb[w];
            eA += se[w][0];
            distinct += se[w][1];
        }
        int64_t *rec = h.part + 4 * slice;
        const i128 g = (i128)best.g;
        __hip_atomic_store(&rec[0], (int64_t)(uint64_t)(u128)g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&rec[1], (int64_t)(g >> 64), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&rec[2], (int64_t)best.c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&rec[3], best.e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int64_t first = h.hoff[p] / HUB_SLICE, nsl = h.hoff[p + 1] / HUB_SLICE - first;
        int64_t *aux = h.aux + 8 * first;
        if (eA) atomicAdd((unsigned long long *)&aux[2], (unsigned long long)eA);
        if (distinct) atomicAdd((unsigned long long *)&aux[3], (unsigned long long)distinct);
        __threadfence();
        const int64_t done = __hip_atomic_fetch_add(&aux[4], (int64_t)1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (done == nsl - 1) {
            __threadfence();
            hub_decide_one<GT>(a, h, p);
        }
    }
}

template <int WK, typename GT>
__global__ __launch_bounds__(BLOCK) void k_sweep_all(SweepArgs a, FusedBins f, HubArgs h)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned long long bstat[5];
    __shared__ int64_t red[BLOCK / 64];
    const int64_t blk = blockIdx.x;
    if (blk >= f.hub_block0) {
        hub_insert_tile<WK>(a, h, blk - f.hub_block0, smem, red);
        return;
    }
    int b = 1;
    while (b < 9 && blk >= f.bins[b + 1].block0) ++b;
    const int64_t tile = blk - f.bins[b].block0;
    switch (b) {
    case 1: sweep_tile<4, WK, GT>(a, f.bins[1], tile, 3, smem, bstat); break;
    case 2: sweep_tile<8, WK, GT>(a, f.bins[2], tile, 4, smem, bstat); break;
    case 3: sweep_tile<16, WK, GT>(a, f.bins[3], tile, 5, smem, bstat); break;
    case 4: sweep_tile<32, WK, GT>(a, f.bins[4], tile, 6, smem, bstat); break;
    case 5: sweep_tile<64, WK, GT>(a, f.bins[5], tile, 7, smem, bstat); break;
    case 6: sweep_tile<64, WK, GT>(a, f.bins[6], tile, 9, smem, bstat); break;
    case 7: sweep_tile<256, WK, GT>(a, f.bins[7], tile, 11, smem, bstat); break;
    case 8: sweep_tile<256, WK, GT>(a, f.bins[8], tile, 12, smem, bstat); break;
    default: mid_hub_tile<WK, GT>(a, f.bins[9], f, tile, smem, bstat); break;
    }
}

// ---- host launchers --------------------------------------------------------
template <typename GT> static void small_t(const SweepArgs &a, const FusedBins &f, int64_t blocks, hipStream_t st)
{
    switch (a.g.wk) {
    case W_UNIT: k_sweep_small<W_UNIT, GT><<<(unsigned)blocks, BLOCK, 512 * 8, st>>>(a, f); break;
    case W_I32: k_sweep_small<W_I32, GT><<<(unsigned)blocks, BLOCK, 512 * 12, st>>>(a, f); break;
    default: k_sweep_small<W_I64, GT><<<(unsigned)blocks, BLOCK, 512 * 12, st>>>(a, f); break;
    }
}

template <typename GT>
static void large_t(const SweepArgs &a, const FusedBins &f, const HubArgs &h, int64_t blocks, hipStream_t st)
{
    const size_t lds = (size_t)HUB_LDS * 12; // 4096 slots: int32 key + 64-bit value
    switch (a.g.wk) {
    case W_UNIT: k_sweep_large<W_UNIT, GT><<<(unsigned)blocks, BLOCK, lds, st>>>(a, f, h); break;
    case W_I32: k_sweep_large<W_I32, GT><<<(unsigned)blocks, BLOCK, lds, st>>>(a, f, h); break;
    default: k_sweep_large<W_I64, GT><<<(unsigned)blocks, BLOCK, lds, st>>>(a, f, h); break;
    }
}

static const int kLanes[10] = {0, 4, 8, 16, 32, 64, 64, 256, 256, 256};

bool sweep_small(const SweepArgs &a, FusedBins f, bool wide, hipStream_t st)
{
    int64_t blocks = 0;
    for (int b = 1; b <= 5; ++b) {
        f.bins[b].block0 = blocks;
        blocks += (f.bins[b].count + BLOCK / kLanes[b] - 1) / (BLOCK / kLanes[b]);
    }
    if (blocks == 0) return false;
    if (wide) small_t<i128>(a, f, blocks, st);
    else small_t<int64_t>(a, f, blocks, st);
    return true;
}

bool sweep_large(const SweepArgs &a, FusedBins f, const HubArgs &h, bool wide, hipStream_t st)
{
    int64_t blocks = 0;
    for (int b = 6; b <= 9; ++b) {
        f.bins[b].block0 = blocks;
        blocks += (f.bins[b].count + BLOCK / kLanes[b] - 1) / (BLOCK / kLanes[b]);
    }
    f.hub_block0 = blocks;
    if (h.e > h.s) blocks += h.n_insert;
    if (blocks == 0) return false;
    if (wide) large_t<i128>(a, f, h, blocks, st);
    else large_t<int64_t>(a, f, h, blocks, st);
    return true;
}

bool sweep_hub_scan(const SweepArgs &a, const HubArgs &h, bool wide, hipStream_t st)
{
    if (h.e <= h.s) return false;
    if (wide) k_hub_scan<i128><<<(unsigned)h.n_scan, BLOCK, 0, st>>>(a, h);
    else k_hub_scan<int64_t><<<(unsigned)h.n_scan, BLOCK, 0, st>>>(a, h);
    return true;
}

template <typename GT>
static void all_t(const SweepArgs &a, const FusedBins &f, const HubArgs &h, int64_t blocks, hipStream_t st)
{
    const size_t lds = (size_t)HUB_LDS * 12;
    switch (a.g.wk) {
    case W_UNIT: k_sweep_all<W_UNIT, GT><<<(unsigned)blocks, BLOCK, lds, st>>>(a, f, h); break;
    case W_I32: k_sweep_all<W_I32, GT><<<(unsigned)blocks, BLOCK, lds, st>>>(a, f, h); break;
    default: k_sweep_all<W_I64, GT><<<(unsigned)blocks, BLOCK, lds, st>>>(a, f, h); break;
    }
}

bool sweep_all(const SweepArgs &a, FusedBins f, const HubArgs &h, bool wide, hipStream_t st)
{
    int64_t blocks = 0;
    for (int b = 1; b <= 9; ++b) {
        f.bins[b].block0 = blocks;
        blocks += (f.bins[b].count + BLOCK / kLanes[b] - 1) / (BLOCK / kLanes[b]);
    }
    f.hub_block0 = blocks;
    if (h.e > h.s) blocks += h.n_insert;
    if (blocks == 0) return false;
    if (wide) all_t<i128>(a, f, h, blocks, st);
    else all_t<int64_t>(a, f, h, blocks, st);
    return true;
}

// ---- binning ----------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_bin_keys(const int64_t *off, int64_t n, const int32_t *group,
                                                    uint64_t *keys, int64_t *vals)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        const int b = degree_bin(off[i + 1] - off[i]);
        keys[i] = ((uint64_t)(group ? group[i] : 0) << 4) | (uint64_t)b;
        vals[i] = i;
    }
}

void bin_keys(const Csr &g, const int32_t *group, uint64_t *keys, int64_t *vals, hipStream_t st)
{
    if (g.n == 0) return;
    unsigned gb = grid_for(g.n, BLOCK * 4);
    if (gb > 65536) gb = 65536;
    k_bin_keys<<<gb, BLOCK, 0, st>>>(g.off, g.n, group, keys, vals);
}

// off[key] = first index of sorted keys whose key is >= key, for key in [0, nkeys]
__global__ __launch_bounds__(BLOCK) void k_key_offsets(const uint64_t *keys, int64_t n, int64_t nkeys, int64_t *off)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i <= n; i += (int64_t)gridDim.x * BLOCK) {
        const int64_t prev = i == 0 ? -1 : (int64_t)keys[i - 1];
        const int64_t cur = i == n ? nkeys : (int64_t)keys[i];
        for (int64_t k = prev + 1; k <= cur; ++k) off[k] = i;
    }
}

void key_offsets(const uint64_t *keys, int64_t n, int64_t nkeys, int64_t *off, hipStream_t st)
{
    unsigned gb = grid_for(n + 1, BLOCK * 4);
    if (gb > 65536) gb = 65536;
    k_key_offsets<<<gb, BLOCK, 0, st>>>(keys, n, nkeys, off);
}

__global__ __launch_bounds__(BLOCK) void k_narrow(const int64_t *vals, int32_t *out, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        out[i] = (int32_t)vals[i];
}

void narrow_ids(const int64_t *vals, int32_t *out, int64_t n, hipStream_t st)
{
    if (n == 0) return;
    unsigned gb = grid_for(n, BLOCK * 4);
    if (gb > 65536) gb = 65536;
    k_narrow<<<gb, BLOCK, 0, st>>>(vals, out, n);
}

__global__ __launch_bounds__(BLOCK) void k_hub_sizes(const int64_t *off, const int32_t *verts, int64_t count,
                                                     int64_t *slots, int64_t *chunks)
{
    for (int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x; p < count; p += (int64_t)gridDim.x * BLOCK) {
        const int32_t v = verts[p];
        const int64_t d = off[v + 1] - off[v];
        const int bin = degree_bin(d);
        slots[p] = bin >= 9 ? pow2_ceil(2 * d) : 0; // >= 8192, a multiple of HUB_SLICE
        chunks[p] = bin == 10 ? (d + HUB_CHUNK - 1) / HUB_CHUNK : 0;
    }
}

void hub_prefix(const Csr &g, const int32_t *verts, int64_t count, int64_t *hoff, int64_t *cpre, int64_t *tmp,
                Scratch &s, hipStream_t st)
{
    if (count == 0) {
        fill<int64_t>(hoff, 0, 1, st);
        fill<int64_t>(cpre, 0, 1, st);
        return;
    }
    unsigned gb = grid_for(count, BLOCK * 4);
    if (gb > 65536) gb = 65536;
    k_hub_sizes<<<gb, BLOCK, 0, st>>>(g.off, verts, count, tmp, cpre);
    scan_i64(tmp, hoff, count, hoff + count, s, st);
    scan_i64(cpre, tmp, count, tmp + count, s, st);  // chunk prefix lands in tmp ...
    hipMemcpyAsync(cpre, tmp, (count + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, st); // ... then cpre
}

__global__ __launch_bounds__(BLOCK) void k_gather_i64(const int64_t *src, const int64_t *idx, int64_t n, int64_t *out)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        out[i] = src[idx[i]];
}

void gather_i64(const int64_t *src, const int64_t *idx, int64_t n, int64_t *out, hipStream_t st)
{
    if (n <= 0) return;
    k_gather_i64<<<grid_for(n, BLOCK), BLOCK, 0, st>>>(src, idx, n, out);
}

// ---- community totals (Eq. 2) for movers ------------------------------------
__global__ __launch_bounds__(BLOCK) void k_commit(const int32_t *verts, int64_t count, int32_t *comm_prev,
                                                  const int32_t *comm_next, const int64_t *k, int64_t *a,
                                                  int32_t *size)
{
    for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < count; t += (int64_t)gridDim.x * BLOCK) {
        const int32_t i = verts ? verts[t] : (int32_t)t;
        const int32_t A = comm_prev[i], B = comm_next[i];
        if (A != B) {
            const int64_t ki = k[i];
            atomicAdd((unsigned long long *)&a[A], (unsigned long long)(-ki));
            atomicAdd((unsigned long long *)&a[B], (unsigned long long)ki);
            atomicSub(&size[A], 1);
            atomicAdd(&size[B], 1);
            comm_prev[i] = B;
        }
    }
}

void commit(const int32_t *verts, int64_t count, int32_t *comm_prev, const int32_t *comm_next, const int64_t *k,
            int64_t *a, int32_t *size, hipStream_t st)
{
    if (count <= 0) return;
    unsigned gc = grid_for(count, BLOCK * 4);
    if (gc > 65536) gc = 65536;
    k_commit<<<gc, BLOCK, 0, st>>>(verts, count, comm_prev, comm_next, k, a, size);
}

void clear_stats(SweepStats *s, int count, hipStream_t st)
{
    fill<int64_t>((int64_t *)s, 0, (int64_t)count * (int64_t)(sizeof(SweepStats) / sizeof(int64_t)), st);
}

} // namespace lv
