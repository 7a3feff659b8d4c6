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

template <int LPV, int WK, typename GT, bool GLOBAL>
__global__ __launch_bounds__(BLOCK) void k_sweep(SweepArgs a, int shift_lds)
{
    typedef typename std::conditional<(WK == W_UNIT && !GLOBAL), uint32_t, unsigned long long>::type VT;
    constexpr int VPB = BLOCK / LPV;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned long long bstat[5];

    const int grp = threadIdx.x / LPV, lane = threadIdx.x % LPV;
    const int64_t vidx = (int64_t)blockIdx.x * VPB + grp;
    const bool valid = vidx < a.count;
    const int32_t i = valid ? a.verts[vidx] : 0;

    int32_t *tkey;
    VT *tval;
    int64_t S;
    int shift;
    if (GLOBAL) {
        const int64_t t0 = valid ? a.hoff[vidx] : 0;
        S = valid ? a.hoff[vidx + 1] - t0 : 0;
        tkey = a.hkey + t0;
        tval = (VT *)(a.hval + t0);
        shift = S > 0 ? (__ffsll((unsigned long long)S) - 1) : 0;
    } else {
        S = (int64_t)1 << shift_lds;
        shift = shift_lds;
        tkey = (int32_t *)smem + grp * S;
        tval = (VT *)(smem + (size_t)VPB * S * sizeof(int32_t)) + grp * S;
        for (int64_t s = lane; s < S; s += LPV) {
            tkey[s] = -1;
            tval[s] = 0;
        }
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
            int32_t cur;
            if (GLOBAL) {
                cur = atomicCAS(&tkey[h], -1, c);
                if (cur == -1 || cur == c) {
                    atomicAdd(&tval[h], (VT)w);
                    break;
                }
            } else {
                cur = tkey[h];
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
            }
            h = (h + 1) & (uint32_t)(S - 1);
        }
    }
    if (GLOBAL) __threadfence();
    __syncthreads();

    // gains over the distinct communities (Eq. 4 scaled by 2m^2), best by (G, -c)
    const int64_t ki = valid ? a.k[i] : 0;
    Best<GT> best{0, -1, 0};
    int64_t eA = 0, distinct = 0;
    for (int64_t s = lane; s < S; s += LPV) {
        int32_t c;
        int64_t e;
        if (GLOBAL) {
            c = __hip_atomic_load(&tkey[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (c < 0) continue;
            e = (int64_t)__hip_atomic_load(&tval[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            tkey[s] = -1; // leave the table clean for the next sweep
            tval[s] = 0;
        } else {
            c = tkey[s];
            if (c < 0) continue;
            e = (int64_t)tval[s];
        }
        ++distinct;
        if (c == A) {
            eA = e;
            continue;
        }
        Best<GT> cand{(GT)a.two_m * (GT)e - (GT)ki * (GT)a.a[c], c, e};
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
    if (lane == 0 && valid) {
        const GT stay = (GT)a.two_m * (GT)eA - (GT)ki * (GT)(a.a[A] - ki);
        bool move = best.c >= 0 && best.g > stay;
        if (move && a.singlet && a.size[A] == 1 && a.size[best.c] == 1 && best.c > A) move = false;
        a.comm_next[i] = move ? best.c : A;
        if (move) {
            atomicAdd(&bstat[0], 1ull);
            atomicAdd(&bstat[2], (unsigned long long)(2 * (best.e - eA)));
        }
        atomicAdd(&bstat[1], (unsigned long long)(eA + wself));
        atomicAdd(&bstat[3], (unsigned long long)distinct);
        atomicAdd(&bstat[4], (unsigned long long)(end - beg));
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        const unsigned long long v = bstat[threadIdx.x];
        if (v) atomicAdd((unsigned long long *)&a.stats->moves + threadIdx.x, v);
    }
}

template <int LPV, bool GLOBAL, typename GT>
static void launch_wk(const SweepArgs &a, int shift, hipStream_t st)
{
    constexpr int VPB = BLOCK / LPV;
    const unsigned grid = grid_for(a.count, VPB);
    size_t lds = 0;
    switch (a.g.wk) {
    case W_UNIT:
        if (!GLOBAL) lds = (size_t)VPB * ((size_t)1 << shift) * (sizeof(int32_t) + sizeof(uint32_t));
        k_sweep<LPV, W_UNIT, GT, GLOBAL><<<grid, BLOCK, lds, st>>>(a, shift);
        break;
    case W_I32:
        if (!GLOBAL) lds = (size_t)VPB * ((size_t)1 << shift) * (sizeof(int32_t) + sizeof(uint64_t));
        k_sweep<LPV, W_I32, GT, GLOBAL><<<grid, BLOCK, lds, st>>>(a, shift);
        break;
    default:
        if (!GLOBAL) lds = (size_t)VPB * ((size_t)1 << shift) * (sizeof(int32_t) + sizeof(uint64_t));
        k_sweep<LPV, W_I64, GT, GLOBAL><<<grid, BLOCK, lds, st>>>(a, shift);
        break;
    }
}

template <typename GT> static void sweep_bin_t(int bin, const SweepArgs &a, hipStream_t st)
{
    switch (bin) {
    case 1: launch_wk<4, false, GT>(a, 3, st); break;     // d <= 4: 8 slots
    case 2: launch_wk<8, false, GT>(a, 4, st); break;     // d <= 8: 16 slots
    case 3: launch_wk<16, false, GT>(a, 5, st); break;    // d <= 16: 32 slots
    case 4: launch_wk<32, false, GT>(a, 6, st); break;    // d <= 32: 64 slots
    case 5: launch_wk<64, false, GT>(a, 7, st); break;    // d <= 64: 128 slots
    case 6: launch_wk<64, false, GT>(a, 9, st); break;    // d <= 256: 512 slots
    case 7: launch_wk<256, false, GT>(a, 11, st); break;  // d <= 1024: 2048 slots
    case 8: launch_wk<256, false, GT>(a, 12, st); break;  // d <= 2048: 4096 slots
    case 9: launch_wk<256, true, GT>(a, 0, st); break;    // hubs: HBM tables
    default: break;
    }
}

void sweep_bin(int bin, const SweepArgs &a, bool wide, hipStream_t st)
{
    if (a.count <= 0) return;
    if (wide) sweep_bin_t<i128>(bin, a, st);
    else sweep_bin_t<int64_t>(bin, a, st);
}

// ---- binning ----------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_bin_keys(const int64_t *off, int64_t n, const int32_t *group,
                                                    uint64_t *keys, int64_t *vals, int32_t *hist)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        const int b = degree_bin(off[i + 1] - off[i]);
        const uint64_t key = ((uint64_t)(group ? group[i] : 0) << 4) | (uint64_t)b;
        keys[i] = key;
        vals[i] = i;
        atomicAdd(&hist[key], 1);
    }
}

void bin_keys(const Csr &g, const int32_t *group, uint64_t *keys, int64_t *vals, int32_t *hist, hipStream_t st)
{
    if (g.n == 0) return;
    unsigned gb = grid_for(g.n, BLOCK * 4);
    if (gb > 65536) gb = 65536;
    k_bin_keys<<<gb, BLOCK, 0, st>>>(g.off, g.n, group, keys, vals, hist);
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
                                                     int64_t *sz)
{
    for (int64_t h = (int64_t)blockIdx.x * BLOCK + threadIdx.x; h < count; h += (int64_t)gridDim.x * BLOCK) {
        const int32_t v = verts[h];
        const int64_t d = off[v + 1] - off[v];
        sz[h] = degree_bin(d) == 9 ? pow2_ceil(2 * d) : 0;
    }
}

int64_t hub_tables(const Csr &g, const int32_t *verts, int64_t count, int64_t *hoff, int64_t *tmp, Scratch &s,
                   hipStream_t st)
{
    if (count == 0) return 0;
    k_hub_sizes<<<grid_for(count, BLOCK), BLOCK, 0, st>>>(g.off, verts, count, tmp);
    scan_i64(tmp, hoff, count, hoff + count, s, st);
    int64_t total = 0;
    hipMemcpyAsync(&total, hoff + count, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    return total;
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
