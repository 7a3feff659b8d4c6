// The synchronous local-moving sweep (Alg. 1 inner loop, Eq. 1, 4, 5 and the
// minimum-label heuristics of Sec. 5.1) as degree-binned gfx950 kernels.
//
// Every vertex of a launch reads only the state of the previous iteration
// (or colour class): comm_prev, a (community degrees) and size.  A group of
// LPV lanes gathers the vertex's row, sums the edge weight per neighbouring
// community e_{i->c} in an open-addressed LDS hash table (rows up to 2048
// entries; longer rows in chunks whose tables are merged per hash bucket by
// a second pass), then evaluates the exact
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

// adds w to community c's slot of an open-addressed LDS table of 2^shift
// slots (linear probing; -1 marks a free slot); the lane that claims the
// slot adds `first` as well
template <typename VT>
__device__ __forceinline__ void table_add(int32_t *tkey, VT *tval, int shift, int32_t c, VT w, VT first = 0)
{
    const uint32_t mask = (1u << shift) - 1;
    uint32_t h = slot_hash(c, shift);
    for (;;) {
        int32_t cur = tkey[h];
        if (cur == c) {
            atomicAdd(&tval[h], w);
            return;
        }
        if (cur == -1) {
            cur = atomicCAS(&tkey[h], -1, c);
            if (cur == -1 || cur == c) {
                atomicAdd(&tval[h], cur == -1 ? w + first : w);
                return;
            }
        }
        h = (h + 1) & mask;
    }
}

// Entries a lane loads (columns, weights, then the neighbours' communities)
// before it inserts any of them: the community gathers are random reads, and
// issuing several before the first is used keeps more of them in flight.
constexpr int GATHER_K = 4;

// Gathers the entries [beg, end) of vertex i, taken by a lane at stride
// `stride` from `first`, into the table; returns the self-loop weight seen.
// PK: the communities come packed with their totals (SweepArgs::cpack), and a
// slot holds e_{i->c} in its low and a_c in its high 32 bits.
template <int WK, typename VT, bool PK = false>
__device__ __forceinline__ int64_t gather_row(const SweepArgs &a, int32_t i, int64_t first, int64_t end, int stride,
                                              int32_t *tkey, VT *tval, int shift)
{
    static_assert(!PK || sizeof(VT) == 8, "a packed slot holds e and a_c");
    int64_t wself = 0;
    for (int64_t e0 = first; e0 < end; e0 += (int64_t)GATHER_K * stride) {
        int32_t c[GATHER_K];
        int64_t w[GATHER_K];
#pragma unroll
        for (int k = 0; k < GATHER_K; ++k) {
            const int64_t e = e0 + (int64_t)k * stride;
            c[k] = -1;
            w[k] = 0;
            if (e < end) {
                const int32_t j = a.g.col[e];
                const int64_t x = WLoad<WK>::at(a.g.w, e);
                if (j == i) wself += x;
                else {
                    c[k] = j;
                    w[k] = x;
                }
            }
        }
        if constexpr (PK) {
            uint64_t p[GATHER_K];
#pragma unroll
            for (int k = 0; k < GATHER_K; ++k) p[k] = c[k] >= 0 ? a.cpack[c[k]] : 0;
#pragma unroll
            for (int k = 0; k < GATHER_K; ++k)
                if (c[k] >= 0)
                    table_add<VT>(tkey, tval, shift, (int32_t)(uint32_t)p[k], (VT)w[k], (VT)(p[k] & ~0xffffffffull));
        } else {
            if (!a.singleton) {
#pragma unroll
                for (int k = 0; k < GATHER_K; ++k)
                    if (c[k] >= 0) c[k] = a.comm_prev[c[k]];
            }
#pragma unroll
            for (int k = 0; k < GATHER_K; ++k)
                if (c[k] >= 0) table_add<VT>(tkey, tval, shift, c[k], (VT)w[k]);
        }
    }
    return wself;
}

// A sweep from the singleton partition (the first of every phase): the
// entries [first, end) of vertex i taken at `stride` are each a candidate of
// their own, C(j) = j with e_{i->j} = w_ij (columns are unique) and a_j = k_j;
// updates the lane's best (G, -j), its self-loop weight and its count of
// distinct candidates.  The degrees of GATHER_K entries are read together.
template <int WK, typename GT>
__device__ __forceinline__ void singleton_row(const SweepArgs &a, int32_t i, int64_t ki, int64_t two_m, int64_t first,
                                              int64_t end, int stride, Best<GT> &best, int64_t &wself,
                                              int64_t &distinct)
{
    for (int64_t e0 = first; e0 < end; e0 += (int64_t)GATHER_K * stride) {
        int32_t j[GATHER_K];
        int64_t w[GATHER_K], kj[GATHER_K];
#pragma unroll
        for (int k = 0; k < GATHER_K; ++k) {
            const int64_t e = e0 + (int64_t)k * stride;
            j[k] = -1;
            w[k] = 0;
            if (e < end) {
                j[k] = a.g.col[e];
                w[k] = WLoad<WK>::at(a.g.w, e);
            }
        }
#pragma unroll
        for (int k = 0; k < GATHER_K; ++k) kj[k] = (j[k] >= 0 && j[k] != i) ? a.a[j[k]] : 0;
#pragma unroll
        for (int k = 0; k < GATHER_K; ++k) {
            if (j[k] < 0) continue;
            if (j[k] == i) {
                wself += w[k];
                continue;
            }
            ++distinct;
            Best<GT> cand{(GT)two_m * (GT)w[k] - (GT)ki * (GT)kj[k], j[k], w[k]};
            if (better(cand, best)) best = cand;
        }
    }
}

// One block-tile of a degree bin: VPB = BLOCK / LPV vertices, LPV lanes each,
// hash tables of 2^shift slots per vertex in LDS.
template <int LPV, int WK, typename GT, bool PK>
__device__ __forceinline__ void sweep_tile(const SweepArgs &a, const BinRange &br, int64_t tile, int shift,
                                           unsigned char *smem, unsigned long long *bstat)
{
    typedef typename std::conditional<WK == W_UNIT && !PK, uint32_t, unsigned long long>::type VT;
    constexpr int VPB = BLOCK / LPV;
    const int grp = threadIdx.x / LPV, lane = threadIdx.x % LPV;
    const int64_t vidx = tile * VPB + grp;
    const int32_t i = vidx < br.count ? br.verts[vidx] : 0;
    const bool valid = vidx < br.count && sweeping(a, i);
    const int64_t two_m = valid ? two_m_of(a, i) : 0;

    const int64_t S = (int64_t)1 << shift;
    int32_t *tkey = (int32_t *)smem + grp * S;
    VT *tval = (VT *)(smem + (size_t)VPB * S * sizeof(int32_t)) + grp * S;
    if (!a.singleton) // a sweep from the singleton partition needs no table
        for (int64_t s = lane; s < S; s += LPV) {
            tkey[s] = -1;
            tval[s] = 0;
        }
    if (threadIdx.x < 5) bstat[threadIdx.x] = 0;
    __syncthreads();

    int64_t beg = 0, end = 0, wself = 0;
    int32_t A = 0;
    if (valid) {
        beg = a.g.off[i];
        end = a.g.off[i + 1];
        A = a.comm_prev[i];
    }
    const int64_t ki = valid ? a.k[i] : 0;
    Best<GT> best{0, -1, 0};
    int64_t eA = 0, distinct = 0;
    if (a.singleton) {
        // every vertex is alone: each non-self neighbour j is a distinct
        // candidate community with e = w_ij and a_j = k_j, and e_A = 0
        if (valid) singleton_row<WK, GT>(a, i, ki, two_m, beg + lane, end, LPV, best, wself, distinct);
    } else {
    // gather: e_{i->c} per neighbouring community (Eq. 1), self-loop apart
    if (valid) wself = gather_row<WK, VT, PK>(a, i, beg + lane, end, LPV, tkey, tval, shift);
    __syncthreads();

    // gains over the distinct communities (Eq. 4 scaled by 2m^2), best by
    // (G, -c); the community degrees of GATHER_K slots are read together
    for (int64_t s0 = lane; s0 < S; s0 += (int64_t)GATHER_K * LPV) {
        int32_t c[GATHER_K];
        int64_t ac[GATHER_K];
#pragma unroll
        for (int k = 0; k < GATHER_K; ++k) {
            const int64_t s = s0 + (int64_t)k * LPV;
            c[k] = s < S ? tkey[s] : -1;
        }
        if constexpr (!PK) {
#pragma unroll
            for (int k = 0; k < GATHER_K; ++k) ac[k] = (c[k] >= 0 && c[k] != A) ? a.a[c[k]] : 0;
        }
#pragma unroll
        for (int k = 0; k < GATHER_K; ++k) {
            if (c[k] < 0) continue;
            int64_t e;
            if constexpr (PK) {
                const uint64_t tv = (uint64_t)tval[s0 + (int64_t)k * LPV];
                e = (int64_t)(tv & 0xffffffffull);
                ac[k] = (int64_t)(tv >> 32);
            } else {
                e = (int64_t)tval[s0 + (int64_t)k * LPV];
            }
            ++distinct;
            if (c[k] == A) {
                eA = e;
                continue;
            }
            Best<GT> cand{(GT)two_m * (GT)e - (GT)ki * (GT)ac[k], c[k], e};
            if (better(cand, best)) best = cand;
        }
    }
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
        if (v) atomicAdd((unsigned long long *)&br.stats[blockIdx.x % STAT_REP].moves + threadIdx.x, v);
    }
}

// hubs: rows longer than 2048 entries -----------------------------------------
// Pass 1 (partition) and pass 2 (aggregate) keep every per-community sum in
// LDS; HBM only carries the chunks' distinct pairs between the passes, so no
// HBM location is updated by more than one workgroup.
constexpr int HUB_T1 = 2 * HUB_CHUNK; // pass-1 table slots (2^11)
constexpr int HUB_T2 = 4096;          // pass-2 table slots (2^12)
constexpr int HUB_CAP2 = 3072;        // distinct keys one pass-2 round may hold
constexpr int HUB_BLOCK2 = 512;
constexpr int HUB_SEGS = 1024;        // chunk segments a pass-2 block stages at a time

// bucket of community c among 2^lp (top bits of the Fibonacci hash)
__device__ __forceinline__ int hub_bucket(int32_t c, int lp)
{
    return lp ? (int)(((uint32_t)c * 0x9E3779B1u) >> (32 - lp)) : 0;
}

// MurmurHash3 finalizer: pass-2 slots (top bits) and rounds (low bits),
// independent of the bucket bits
__device__ __forceinline__ uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

// exclusive scan of x[0, len) in LDS by NT threads (len <= K * NT); x[len] = total
template <int NT, int K> __device__ __forceinline__ void lds_exscan(int32_t *x, int len, int32_t *wsum)
{
    const int t = threadIdx.x;
    int32_t v[K], s = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = K * t + k;
        v[k] = i < len ? x[i] : 0;
        s += v[k];
    }
    int32_t inc = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(inc, o, 64);
        if ((t & 63) >= o) inc += y;
    }
    if ((t & 63) == 63) wsum[t >> 6] = inc;
    __syncthreads();
    int32_t run = inc - s, tot = 0;
    for (int w = 0; w < NT / 64; ++w) {
        if (w < (t >> 6)) run += wsum[w];
        tot += wsum[w];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = K * t + k;
        if (i < len) x[i] = run;
        run += v[k];
    }
    if (t == 0) x[len] = tot;
    __syncthreads();
}

// LDS bytes of a pass-1 block
template <typename VT> constexpr size_t hub_part_lds()
{
    return (size_t)HUB_T1 * (sizeof(int32_t) + sizeof(VT)) + sizeof(int32_t) * (HUB_PMAX + 1);
}

template <int WK, typename VT>
__device__ __forceinline__ void hub_part_tile(const SweepArgs &a, const HubArgs &h, int64_t tile, unsigned char *smem)
{
    __shared__ int32_t wsum[BLOCK / 64];
    int32_t *tkey = (int32_t *)smem;
    VT *tval = (VT *)(smem + HUB_T1 * sizeof(int32_t));
    int32_t *hist = (int32_t *)(smem + HUB_T1 * (sizeof(int32_t) + sizeof(VT)));
    const int64_t target = h.chunk0 + tile;
    const HubChunk ck = h.chunks[target];
    const int32_t v = ck.v;
    if (!sweeping(a, v)) return; // uniform over the block
    const int64_t beg = ck.beg, end = ck.end;
    const int P = ck.P;
    const int lp = __ffs(P) - 1;
    for (int s = threadIdx.x; s < HUB_T1; s += BLOCK) {
        tkey[s] = -1;
        tval[s] = 0;
    }
    for (int b = threadIdx.x; b <= P; b += BLOCK) hist[b] = 0;
    __syncthreads();
    {
        // the only chunk holding the self-loop leaves it for the decision
        const int64_t wself = gather_row<WK, VT>(a, v, beg + threadIdx.x, end, BLOCK, tkey, tval, 11);
        static_assert(HUB_T1 == 1 << 11, "pass-1 table of 2^11 slots");
        if (wself) h.self[ck.self_slot] = wself;
    }
    __syncthreads();
    // rank of every distinct community inside its bucket, then bucket starts
    constexpr int PER = HUB_T1 / BLOCK;
    int32_t rk[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int32_t c = tkey[threadIdx.x + j * BLOCK];
        rk[j] = c >= 0 ? atomicAdd(&hist[hub_bucket(c, lp)], 1) : 0;
    }
    __syncthreads();
    lds_exscan<BLOCK, 4>(hist, P, wsum);
    const int64_t base = target * HUB_CHUNK;
    VT *pval = (VT *)h.pval;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int s = threadIdx.x + j * BLOCK;
        const int32_t c = tkey[s];
        if (c < 0) continue;
        const int64_t at = base + hist[hub_bucket(c, lp)] + rk[j];
        h.pkey[at] = c;
        pval[at] = tval[s];
    }
    int32_t *bo = h.boff + ck.bo;
    for (int b = threadIdx.x; b <= P; b += BLOCK) bo[b] = hist[b];
}

// one tile of bin b with the bin's lanes per vertex (a launch-time choice
// among kLaneChoices[b]); every (bin, lanes) pair is its own instance, so the
// table size stays a compile-time constant.  LO..HI: the bins the launch has.
template <int WK, typename GT, int LO, int HI, bool PK = false>
__device__ __forceinline__ void bin_tile(const SweepArgs &a, const FusedBins &f, int b, int64_t tile,
                                         unsigned char *smem, unsigned long long *bstat)
{
    const BinRange &br = f.bins[b];
    const int l = f.lanes[b];
#define LV_TILE(B, L, SH)                                                                                              \
    if ((B) >= LO && (B) <= HI && b == (B) && l == (L)) {                                                             \
        sweep_tile<L, WK, GT, PK>(a, br, tile, SH, smem, bstat);                                                       \
        return;                                                                                                        \
    }
    LV_TILE(1, 4, 3) LV_TILE(1, 8, 3)
    LV_TILE(2, 8, 4) LV_TILE(2, 4, 4) LV_TILE(2, 16, 4)
    LV_TILE(3, 16, 5) LV_TILE(3, 8, 5) LV_TILE(3, 32, 5)
    LV_TILE(4, 32, 6) LV_TILE(4, 16, 6) LV_TILE(4, 64, 6)
    LV_TILE(5, 64, 7) LV_TILE(5, 32, 7)
    LV_TILE(6, 64, 9) LV_TILE(6, 256, 9)
    LV_TILE(7, 256, 11)
    LV_TILE(8, 256, 12)
#undef LV_TILE
}

// Fused launches: blocks are assigned to bins by block ranges.
//  small: bins 1..5 (4..64 lanes per vertex, 512 LDS slots per block)
//  large: bins 6..7 (64 or 256 lanes per vertex, up to 2048 slots) and hub pass 1
//  bin 8: 256 lanes per vertex, 4096 slots, alone (its 48 KB tables would cap
//         the large launch at three workgroups per CU; measured on R-MAT 24,
//         the split took the plain sweeps' large launches from 6.7 to 4.8 ms)
template <int WK, typename GT, bool PK>
__global__ __launch_bounds__(BLOCK) void k_sweep_small(SweepArgs a, FusedBins f)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned long long bstat[5];
    const int64_t blk = blockIdx.x;
    int b = 1;
    while (b < 5 && blk >= f.bins[b + 1].block0) ++b;
    bin_tile<WK, GT, 1, 5, PK>(a, f, b, blk - f.bins[b].block0, smem, bstat);
}

template <int WK, typename GT, typename VT, bool PK>
__global__ __launch_bounds__(BLOCK) void k_sweep_large(SweepArgs a, FusedBins f, HubArgs h)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned long long bstat[5];
    const int64_t blk = blockIdx.x;
    if (blk >= f.hub_block0) {
        hub_part_tile<WK, VT>(a, h, blk - f.hub_block0, smem);
        return;
    }
    const int b = blk >= f.bins[7].block0 ? 7 : 6;
    bin_tile<WK, GT, 6, 7, PK>(a, f, b, blk - f.bins[b].block0, smem, bstat);
}

// bin 8 alone (rows of 1,025-2,048 entries, 4,096-slot tables): its LDS
// would otherwise set the occupancy of the large launch's other tiles
template <int WK, typename GT, bool PK>
__global__ __launch_bounds__(BLOCK) void k_sweep_bin8(SweepArgs a, FusedBins f)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned long long bstat[5];
    bin_tile<WK, GT, 8, 8, PK>(a, f, 8, blockIdx.x, smem, bstat);
}

template <int WK, typename GT, typename VT>
__global__ __launch_bounds__(BLOCK) void k_sweep_all(SweepArgs a, FusedBins f, HubArgs h)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned long long bstat[5];
    const int64_t blk = blockIdx.x;
    if (blk >= f.hub_block0) {
        hub_part_tile<WK, VT>(a, h, blk - f.hub_block0, smem);
        return;
    }
    int b = 1;
    while (b < 8 && blk >= f.bins[b + 1].block0) ++b;
    bin_tile<WK, GT, 1, 8>(a, f, b, blk - f.bins[b].block0, smem, bstat);
}

// decision of hub p from its bucket records and self-loop slot, by one
// wavefront (lanes read the records in parallel); reads no community state
// (the records carry what the rule needs), so it may run while other
// vertices of its class are being committed.  Returns the decision to all
// lanes.
template <typename GT> __device__ __forceinline__ int32_t hub_decide(const SweepArgs &a, const HubArgs &h, int64_t p)
{
    const int lane = threadIdx.x & 63;
    const int32_t v = h.verts[p];
    const int32_t A = a.comm_prev[v];
    const int64_t q0 = h.bpre[p], q1 = h.bpre[p + 1];
    Best<GT> best{0, -1, 0};
    int64_t eA = 0, distinct = 0, size_best = 0;
    for (int64_t q = q0 + lane; q < q1; q += 64) {
        const int64_t *rec = h.part + HUB_REC * q;
        const i128 g = (i128)(((u128)(uint64_t)rec[1] << 64) | (u128)(uint64_t)rec[0]);
        Best<GT> cand{(GT)g, (int32_t)rec[2], rec[3]};
        if (better(cand, best)) {
            best = cand;
            size_best = rec[6];
        }
        eA += rec[4];
        distinct += rec[5];
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        Best<GT> o;
        o.g = shfl_xor_t(best.g, m, 64);
        o.c = shfl_xor_t(best.c, m, 64);
        o.e = shfl_xor_t(best.e, m, 64);
        const int64_t os = shfl_xor_t(size_best, m, 64);
        if (better(o, best)) {
            best = o;
            size_best = os;
        }
        eA += shfl_xor_t(eA, m, 64);
        distinct += shfl_xor_t(distinct, m, 64);
    }
    const int64_t *rec0 = h.part + HUB_REC * q0;
    const int64_t aA = rec0[7], sizeA = rec0[8];
    const int64_t wself = h.self[q0];
    const int64_t kv = a.k[v];
    const GT stay = (GT)two_m_of(a, v) * (GT)eA - (GT)kv * (GT)(aA - kv);
    bool move = best.c >= 0 && best.g > stay;
    if (move && a.singlet && sizeA == 1 && size_best == 1 && best.c > A) move = false;
    const int32_t dest = move ? best.c : A;
    if (lane == 0) {
        h.self[q0] = 0;
        a.comm_next[v] = dest;
        unsigned long long *st = a.gid ? (unsigned long long *)&a.gstats[8 * (int64_t)a.gid[v]]
                                       : (unsigned long long *)&a.stats[p % STAT_REP].moves;
        if (move) {
            atomicAdd(&st[0], 1ull);
            atomicAdd(&st[2], (unsigned long long)(2 * (best.e - eA)));
        }
        atomicAdd(&st[1], (unsigned long long)(eA + wself));
        atomicAdd(&st[3], (unsigned long long)distinct);
        atomicAdd(&st[4], (unsigned long long)(a.g.off[v + 1] - a.g.off[v]));
    }
    return dest;
}

// Hub rows in a sweep from the singleton partition: every neighbour is a
// community of its own, so nothing is aggregated and pass 1 is not run.
// One block per (hub, bucket) scans the bucket's equal slice of the hub's
// row and writes the slice's best (G, -j) and counts in the bucket record
// that the decision reads; the slice holding the self-loop stores it at the
// hub's first bucket.
template <int WK, typename GT>
__global__ __launch_bounds__(HUB_BLOCK2) void k_hub_first(SweepArgs a, HubArgs h)
{
    __shared__ Best<GT> sb[HUB_BLOCK2 / 64];
    __shared__ int64_t se[HUB_BLOCK2 / 64][2];
    const int64_t q = h.bucket0 + blockIdx.x;
    const HubBucket bk = h.buckets[q];
    const int32_t v = bk.v;
    if (!sweeping(a, v)) return; // uniform over the block
    const int64_t beg = a.g.off[v], d = a.g.off[v + 1] - beg;
    const int64_t lo = beg + d * bk.b / bk.P, hi = beg + d * (bk.b + 1) / bk.P;
    const int64_t two_m = two_m_of(a, v), kv = a.k[v];
    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    Best<GT> best{0, -1, 0};
    int64_t wself = 0, distinct = 0;
    singleton_row<WK, GT>(a, v, kv, two_m, lo + tid, hi, HUB_BLOCK2, best, wself, distinct);
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        Best<GT> o;
        o.g = shfl_xor_t(best.g, m, 64);
        o.c = shfl_xor_t(best.c, m, 64);
        o.e = shfl_xor_t(best.e, m, 64);
        if (better(o, best)) best = o;
        wself += shfl_xor_t(wself, m, 64);
        distinct += shfl_xor_t(distinct, m, 64);
    }
    if (lane == 0) {
        sb[wid] = best;
        se[wid][0] = wself;
        se[wid][1] = distinct;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < HUB_BLOCK2 / 64; ++w) {
            if (better(sb[w], best)) best = sb[w];
            wself += se[w][0];
            distinct += se[w][1];
        }
        int64_t *rec = h.part + HUB_REC * q;
        const i128 g = (i128)best.g;
        const int32_t A = a.comm_prev[v];
        rec[0] = (int64_t)(uint64_t)(u128)g;
        rec[1] = (int64_t)(g >> 64);
        rec[2] = (int64_t)best.c;
        rec[3] = best.e;
        rec[4] = 0; // e_A: no neighbour shares the hub's one-vertex community
        rec[5] = distinct;
        rec[6] = best.c >= 0 ? a.size[best.c] : 0;
        rec[7] = a.a[A];
        rec[8] = a.size[A];
        if (wself) h.self[q - bk.b] = wself;
    }
}

// one wavefront per hub
template <typename GT> __global__ __launch_bounds__(BLOCK) void k_hub_decide(SweepArgs a, HubArgs h)
{
    const int64_t nw = (int64_t)gridDim.x * (BLOCK / 64);
    for (int64_t p = h.s + (int64_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6); p < h.e; p += nw)
        if (sweeping(a, h.verts[p])) hub_decide<GT>(a, h, p);
}

// Pass 2: one block per (hub, bucket).  The bucket's pairs from every chunk
// of the hub are summed in an LDS table of HUB_T2 slots.  A round holds at
// most HUB_CAP2 distinct communities; if a bucket has more, it is redone in
// R = 2, 4, ... rounds, each taking the communities whose hash has low bits r
// (and, past R = 2^16, in rounds over id ranges of 2048, which always fit).
template <typename GT, typename VT>
__global__ __launch_bounds__(HUB_BLOCK2) void k_hub_agg(SweepArgs a, HubArgs h)
{
    __shared__ int32_t tkey[HUB_T2];
    __shared__ VT tval[HUB_T2];
    __shared__ int32_t s_cnt, s_over;
    __shared__ int32_t seg_lo[HUB_SEGS], seg_pre[HUB_SEGS + 1];
    __shared__ int32_t wsum[HUB_BLOCK2 / 64];
    __shared__ Best<GT> sb[HUB_BLOCK2 / 64];
    __shared__ int64_t se[HUB_BLOCK2 / 64][2];
    const int64_t q = h.bucket0 + blockIdx.x;
    const HubBucket bk = h.buckets[q];
    const int32_t v = bk.v;
    if (!sweeping(a, v)) return; // uniform over the block
    const int P = bk.P;
    const int b = bk.b;
    const int64_t c0 = bk.c0, nch = bk.nch;
    const int32_t *bo = h.boff + bk.xo;
    const VT *pval = (const VT *)h.pval;
    const int32_t A = a.comm_prev[v];
    const int64_t two_m = two_m_of(a, v), kv = a.k[v];
    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    constexpr int NW = HUB_BLOCK2 / 64;
    Best<GT> best{0, -1, 0};
    int64_t eA = 0, distinct = 0;
    for (int64_t R = 1;; R <<= 1) {
        const bool by_range = R > (1 << 16);
        const int64_t rounds = by_range ? ((int64_t)a.g.n + 2047) / 2048 : R;
        bool over = false;
        best = Best<GT>{0, -1, 0};
        eA = 0;
        distinct = 0;
        for (int64_t r = 0; r < rounds && !over; ++r) {
            for (int s = tid; s < HUB_T2; s += HUB_BLOCK2) {
                tkey[s] = -1;
                tval[s] = 0;
            }
            if (tid == 0) {
                s_cnt = 0;
                s_over = 0;
            }
            __syncthreads();
            // the bucket's segments of up to HUB_SEGS chunks at a time, as one
            // flat range over the threads
            for (int64_t cb = 0; cb < nch; cb += HUB_SEGS) {
                const int nb = (int)min((int64_t)HUB_SEGS, nch - cb);
                for (int k = tid; k < nb; k += HUB_BLOCK2) {
                    const int32_t *bk = bo + (cb + k) * (P + 1) + b;
                    seg_lo[k] = bk[0];
                    seg_pre[k] = bk[1] - bk[0];
                }
                __syncthreads();
                lds_exscan<HUB_BLOCK2, HUB_SEGS / HUB_BLOCK2>(seg_pre, nb, wsum);
                const int32_t total = seg_pre[nb];
                for (int32_t t = tid; t < total; t += HUB_BLOCK2) {
                    int lo = 0, hi = nb; // largest k with seg_pre[k] <= t
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (seg_pre[mid] <= t) lo = mid; else hi = mid;
                    }
                    const int64_t at = (c0 + cb + lo) * HUB_CHUNK + seg_lo[lo] + (t - seg_pre[lo]);
                    const int32_t c = h.pkey[at];
                    const uint32_t hc = fmix32((uint32_t)c);
                    if (by_range ? (int64_t)(c >> 11) != r : (int64_t)(hc & (uint32_t)(R - 1)) != r) continue;
                    const VT w = pval[at];
                    uint32_t slot = hc >> 20; // top 12 bits: HUB_T2 slots
                    for (;;) {
                        int32_t cur = tkey[slot];
                        if (cur == c) {
                            atomicAdd(&tval[slot], w);
                            break;
                        }
                        if (cur == -1) {
                            // reserve room first: occupied slots never exceed HUB_CAP2 < HUB_T2,
                            // so every probe sequence meets an empty slot
                            if (atomicAdd(&s_cnt, 1) >= HUB_CAP2) {
                                s_over = 1;
                                break;
                            }
                            cur = atomicCAS(&tkey[slot], -1, c);
                            if (cur == -1) {
                                atomicAdd(&tval[slot], w);
                                break;
                            }
                            atomicSub(&s_cnt, 1);
                            if (cur == c) {
                                atomicAdd(&tval[slot], w);
                                break;
                            }
                        }
                        slot = (slot + 1) & (HUB_T2 - 1);
                    }
                }
                __syncthreads(); // segment arrays are rewritten by the next batch
            }
            __syncthreads();
            const bool ov = s_over != 0;
            if (!ov) {
                static_assert(HUB_T2 % (GATHER_K * HUB_BLOCK2) == 0, "whole slot groups");
                for (int s0 = tid; s0 < HUB_T2; s0 += GATHER_K * HUB_BLOCK2) {
                    int32_t c[GATHER_K];
                    int64_t ac[GATHER_K];
#pragma unroll
                    for (int k = 0; k < GATHER_K; ++k) c[k] = tkey[s0 + k * HUB_BLOCK2];
#pragma unroll
                    for (int k = 0; k < GATHER_K; ++k) ac[k] = (c[k] >= 0 && c[k] != A) ? a.a[c[k]] : 0;
#pragma unroll
                    for (int k = 0; k < GATHER_K; ++k) {
                        if (c[k] < 0) continue;
                        const int64_t e = (int64_t)tval[s0 + k * HUB_BLOCK2];
                        ++distinct;
                        if (c[k] == A) {
                            eA += e;
                            continue;
                        }
                        Best<GT> cand{(GT)two_m * (GT)e - (GT)kv * (GT)ac[k], c[k], e};
                        if (better(cand, best)) best = cand;
                    }
                }
            }
            __syncthreads(); // table and flag are read by all before the next round clears them
            over = ov;
        }
        if (!over) break;
    }
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
    if (lane == 0) {
        sb[wid] = best;
        se[wid][0] = eA;
        se[wid][1] = distinct;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < NW; ++w) {
            if (better(sb[w], best)) best = sb[w];
            eA += se[w][0];
            distinct += se[w][1];
        }
        int64_t *rec = h.part + HUB_REC * q;
        const i128 g = (i128)best.g;
        rec[0] = (int64_t)(uint64_t)(u128)g;
        rec[1] = (int64_t)(g >> 64);
        rec[2] = (int64_t)best.c;
        rec[3] = best.e;
        rec[4] = eA;
        rec[5] = distinct;
        rec[6] = best.c >= 0 ? a.size[best.c] : 0;
        rec[7] = a.a[A];
        rec[8] = a.size[A];
    }
}

// ---- host launchers --------------------------------------------------------
// bytes of a table slot: community + e (+ a_c when packed)
static size_t slot_bytes(int wk, bool pk) { return wk == W_UNIT && !pk ? 8 : 12; }

// LDS of bins 1..5 of a launch: vertices per block x table slots x slot bytes
static size_t small_lds(const FusedBins &f, int wk, bool pk)
{
    size_t m = 0;
    for (int b = 1; b <= 5; ++b) {
        const size_t v = (size_t)(BLOCK / f.lanes[b]) << kBinShift[b];
        if (v > m) m = v;
    }
    return m * slot_bytes(wk, pk);
}

template <typename GT, bool PK>
static void small_t(const SweepArgs &a, const FusedBins &f, int64_t blocks, hipStream_t st)
{
    const size_t lds = small_lds(f, a.g.wk, PK);
    switch (a.g.wk) {
    case W_UNIT: k_sweep_small<W_UNIT, GT, PK><<<(unsigned)blocks, BLOCK, lds, st>>>(a, f); break;
    case W_I32: k_sweep_small<W_I32, GT, PK><<<(unsigned)blocks, BLOCK, lds, st>>>(a, f); break;
    default: k_sweep_small<W_I64, GT, PK><<<(unsigned)blocks, BLOCK, lds, st>>>(a, f); break;
    }
}

// dynamic LDS of a fused launch with bins up to 8 and hub pass 1
// dynamic LDS of a launch: the largest table among the bins lo..hi it has
// vertices of, and hub pass 1 if it has hub tiles
static size_t bins_lds(const FusedBins &f, int wk, bool pk, int lo, int hi)
{
    size_t m = 0;
    for (int b = lo; b <= hi; ++b) {
        if (f.bins[b].count == 0) continue;
        const size_t v = ((size_t)(BLOCK / f.lanes[b]) << kBinShift[b]) * slot_bytes(wk, pk);
        if (v > m) m = v;
    }
    return m;
}

template <int WK, typename VT> static size_t fused_lds(const FusedBins &f, bool pk, int hi, bool hubs)
{
    const size_t m = bins_lds(f, WK, pk, 1, hi);
    return hubs && hub_part_lds<VT>() > m ? hub_part_lds<VT>() : m;
}

template <bool ALL, int WK, typename GT, typename VT, bool PK>
static void fused_launch(const SweepArgs &a, const FusedBins &f, const HubArgs &h, int64_t blocks, hipStream_t st)
{
    const size_t lds = fused_lds<WK, VT>(f, PK, ALL ? 8 : 7, blocks > f.hub_block0);
    if constexpr (ALL) k_sweep_all<WK, GT, VT><<<(unsigned)blocks, BLOCK, lds, st>>>(a, f, h);
    else k_sweep_large<WK, GT, VT, PK><<<(unsigned)blocks, BLOCK, lds, st>>>(a, f, h);
}

template <bool ALL, typename GT, typename VT, bool PK = false>
static void fused_t(const SweepArgs &a, const FusedBins &f, const HubArgs &h, int64_t blocks, hipStream_t st)
{
    switch (a.g.wk) {
    case W_UNIT: fused_launch<ALL, W_UNIT, GT, VT, PK>(a, f, h, blocks, st); break;
    case W_I32: fused_launch<ALL, W_I32, GT, VT, PK>(a, f, h, blocks, st); break;
    default: fused_launch<ALL, W_I64, GT, VT, PK>(a, f, h, blocks, st); break;
    }
}

template <bool ALL>
static void fused(const SweepArgs &a, const FusedBins &f, const HubArgs &h, int64_t blocks, bool wide, bool narrow,
                  hipStream_t st)
{
    if (wide) {
        if (narrow) fused_t<ALL, i128, uint32_t>(a, f, h, blocks, st);
        else fused_t<ALL, i128, unsigned long long>(a, f, h, blocks, st);
    } else {
        if (narrow) fused_t<ALL, int64_t, uint32_t>(a, f, h, blocks, st);
        else fused_t<ALL, int64_t, unsigned long long>(a, f, h, blocks, st);
    }
}


// the packed instances: a plain sweep whose 2m fits 32 bits (then the gains
// fit int64 and hub sums fit 32 bits)
static bool packed(const SweepArgs &a, bool wide)
{
    return a.cpack && !a.singleton && !a.gid && !wide && a.two_m <= (int64_t)UINT32_MAX;
}

__global__ __launch_bounds__(BLOCK) void k_pack_communities(const int32_t *comm, const int64_t *a, int64_t n,
                                                            uint64_t *out)
{
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < n; j += (int64_t)gridDim.x * BLOCK) {
        const int32_t c = comm[j];
        out[j] = (uint64_t)(uint32_t)c | ((uint64_t)a[c] << 32);
    }
}

void pack_communities(const int32_t *comm, const int64_t *a, int64_t n, uint64_t *out, hipStream_t st)
{
    if (n <= 0) return;
    unsigned gb = grid_for(n, BLOCK * 4);
    if (gb > 65536) gb = 65536;
    k_pack_communities<<<gb, BLOCK, 0, st>>>(comm, a, n, out);
}

bool sweep_small(const SweepArgs &a, FusedBins f, bool wide, hipStream_t st)
{
    int64_t blocks = 0;
    for (int b = 1; b <= 5; ++b) {
        f.bins[b].block0 = blocks;
        blocks += (f.bins[b].count + BLOCK / f.lanes[b] - 1) / (BLOCK / f.lanes[b]);
    }
    if (blocks == 0) return false;
    if (packed(a, wide)) small_t<int64_t, true>(a, f, blocks, st);
    else if (wide) small_t<i128, false>(a, f, blocks, st);
    else small_t<int64_t, false>(a, f, blocks, st);
    return true;
}

template <typename GT, bool PK>
static void bin8_t(const SweepArgs &a, const FusedBins &f, int64_t blocks, hipStream_t st)
{
    const size_t lds = bins_lds(f, a.g.wk, PK, 8, 8);
    switch (a.g.wk) {
    case W_UNIT: k_sweep_bin8<W_UNIT, GT, PK><<<(unsigned)blocks, BLOCK, lds, st>>>(a, f); break;
    case W_I32: k_sweep_bin8<W_I32, GT, PK><<<(unsigned)blocks, BLOCK, lds, st>>>(a, f); break;
    default: k_sweep_bin8<W_I64, GT, PK><<<(unsigned)blocks, BLOCK, lds, st>>>(a, f); break;
    }
}

bool sweep_bin8(const SweepArgs &a, const FusedBins &f, bool wide, bool narrow, hipStream_t st)
{
    const int64_t blocks = (f.bins[8].count + BLOCK / f.lanes[8] - 1) / (BLOCK / f.lanes[8]);
    if (blocks == 0) return false;
    if (packed(a, wide) && narrow) bin8_t<int64_t, true>(a, f, blocks, st);
    else if (wide) bin8_t<i128, false>(a, f, blocks, st);
    else bin8_t<int64_t, false>(a, f, blocks, st);
    return true;
}

bool sweep_large(const SweepArgs &a, FusedBins f, const HubArgs &h, bool wide, bool narrow, hipStream_t st)
{
    int64_t blocks = 0;
    for (int b = 6; b <= 7; ++b) {
        f.bins[b].block0 = blocks;
        blocks += (f.bins[b].count + BLOCK / f.lanes[b] - 1) / (BLOCK / f.lanes[b]);
    }
    f.bins[8].block0 = blocks; // bin 8 has a launch of its own
    f.bins[8].count = 0;
    f.hub_block0 = blocks;
    if (h.e > h.s && !a.singleton) blocks += h.n_chunks; // from singletons the hubs need no pass 1
    if (blocks == 0) return false;
    if (packed(a, wide) && narrow) fused_t<false, int64_t, uint32_t, true>(a, f, h, blocks, st);
    else fused<false>(a, f, h, blocks, wide, narrow, st);
    return true;
}

bool sweep_all(const SweepArgs &a, FusedBins f, const HubArgs &h, bool wide, bool narrow, hipStream_t st)
{
    int64_t blocks = 0;
    for (int b = 1; b <= 8; ++b) {
        f.bins[b].block0 = blocks;
        blocks += (f.bins[b].count + BLOCK / f.lanes[b] - 1) / (BLOCK / f.lanes[b]);
    }
    f.hub_block0 = blocks;
    if (h.e > h.s && !a.singleton) blocks += h.n_chunks;
    if (blocks == 0) return false;
    fused<true>(a, f, h, blocks, wide, narrow, st);
    return true;
}

bool sweep_hub_agg(const SweepArgs &a, const HubArgs &h, bool wide, bool narrow, bool decide, hipStream_t st)
{
    if (h.e <= h.s || h.n_buckets == 0) return false;
    const unsigned g = (unsigned)h.n_buckets;
    unsigned gd = grid_for(h.e - h.s, BLOCK / 64);
    if (gd > 1024) gd = 1024;
    if (a.singleton) {
        // from singletons: the buckets' slices are scanned directly
#define LV_FIRST(GT)                                                                                                   \
        switch (a.g.wk) {                                                                                              \
        case W_UNIT: k_hub_first<W_UNIT, GT><<<g, HUB_BLOCK2, 0, st>>>(a, h); break;                                  \
        case W_I32: k_hub_first<W_I32, GT><<<g, HUB_BLOCK2, 0, st>>>(a, h); break;                                    \
        default: k_hub_first<W_I64, GT><<<g, HUB_BLOCK2, 0, st>>>(a, h); break;                                       \
        }                                                                                                              \
        if (decide) k_hub_decide<GT><<<gd, BLOCK, 0, st>>>(a, h);
        if (wide) {
            LV_FIRST(i128)
        } else {
            LV_FIRST(int64_t)
        }
#undef LV_FIRST
        return true;
    }
    if (wide) {
        if (narrow) k_hub_agg<i128, uint32_t><<<g, HUB_BLOCK2, 0, st>>>(a, h);
        else k_hub_agg<i128, unsigned long long><<<g, HUB_BLOCK2, 0, st>>>(a, h);
        if (decide) k_hub_decide<i128><<<gd, BLOCK, 0, st>>>(a, h);
    } else {
        if (narrow) k_hub_agg<int64_t, uint32_t><<<g, HUB_BLOCK2, 0, st>>>(a, h);
        else k_hub_agg<int64_t, unsigned long long><<<g, HUB_BLOCK2, 0, st>>>(a, h);
        if (decide) k_hub_decide<int64_t><<<gd, BLOCK, 0, st>>>(a, h);
    }
    return true;
}

// ---- binning ----------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_bin_keys(const int64_t *off, int64_t n, const int32_t *group,
                                                    uint64_t *keys, int64_t *vals, const int32_t *gid,
                                                    const int32_t *active)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        const int b = (gid && !active[gid[i]]) ? 0 : degree_bin(off[i + 1] - off[i]);
        keys[i] = ((uint64_t)(group ? group[i] : 0) << 4) | (uint64_t)b;
        vals[i] = i;
    }
}

void bin_keys(const Csr &g, const int32_t *group, uint64_t *keys, int64_t *vals, hipStream_t st, const int32_t *gid,
              const int32_t *active)
{
    if (g.n == 0) return;
    unsigned gb = grid_for(g.n, BLOCK * 4);
    if (gb > 65536) gb = 65536;
    k_bin_keys<<<gb, BLOCK, 0, st>>>(g.off, g.n, group, keys, vals, gid, active);
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
                                                     int64_t *chunks, int64_t *buckets, int64_t *bounds)
{
    for (int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x; p < count; p += (int64_t)gridDim.x * BLOCK) {
        const int32_t v = verts[p];
        const int64_t d = off[v + 1] - off[v];
        const bool hub = degree_bin(d) >= 9;
        const int64_t c = hub ? (d + HUB_CHUNK - 1) / HUB_CHUNK : 0;
        const int64_t P = hub ? hub_buckets(d) : 0;
        chunks[p] = c;
        buckets[p] = P;
        bounds[p] = c * (P + 1);
    }
}

void hub_prefix(const Csr &g, const int32_t *verts, int64_t count, int64_t *cpre, int64_t *bpre, int64_t *xpre,
                Scratch &s, hipStream_t st)
{
    if (count == 0) {
        fill<int64_t>(cpre, 0, 1, st);
        fill<int64_t>(bpre, 0, 1, st);
        fill<int64_t>(xpre, 0, 1, st);
        return;
    }
    unsigned gb = grid_for(count, BLOCK * 4);
    if (gb > 65536) gb = 65536;
    k_hub_sizes<<<gb, BLOCK, 0, st>>>(g.off, verts, count, cpre, bpre, xpre);
    // in place: each scan block reads its own tile before writing it
    scan_i64(cpre, cpre, count, cpre + count, s, st);
    scan_i64(bpre, bpre, count, bpre + count, s, st);
    scan_i64(xpre, xpre, count, xpre + count, s, st);
}


__global__ __launch_bounds__(BLOCK) void k_hub_owners(const int32_t *verts, const int64_t *off, const int64_t *cpre,
                                                      const int64_t *bpre, const int64_t *xpre, int64_t count,
                                                      HubChunk *chunks, HubBucket *buckets)
{
    for (int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x; p < count; p += (int64_t)gridDim.x * BLOCK) {
        const int64_t c0 = cpre[p], c1 = cpre[p + 1];
        if (c1 == c0) continue; // not a hub
        const int32_t v = verts[p];
        const int64_t rb = off[v], re = off[v + 1];
        const int64_t q0 = bpre[p], q1 = bpre[p + 1];
        const int32_t P = (int32_t)(q1 - q0);
        for (int64_t c = c0; c < c1; ++c) {
            HubChunk k;
            k.v = v;
            k.P = P;
            k.beg = rb + (c - c0) * HUB_CHUNK;
            k.end = min(re, k.beg + HUB_CHUNK);
            k.bo = xpre[p] + (c - c0) * (P + 1);
            k.self_slot = q0;
            k.pad = 0;
            chunks[c] = k;
        }
        for (int64_t q = q0; q < q1; ++q) {
            HubBucket k;
            k.v = v;
            k.P = P;
            k.b = (int32_t)(q - q0);
            k.pad = 0;
            k.c0 = c0;
            k.nch = c1 - c0;
            k.xo = xpre[p];
            k.pad2 = 0;
            buckets[q] = k;
        }
    }
}

void hub_owners(const int32_t *verts, const int64_t *off, const int64_t *cpre, const int64_t *bpre,
                const int64_t *xpre, int64_t count, HubChunk *chunks, HubBucket *buckets, hipStream_t st)
{
    if (count <= 0) return;
    unsigned gb = grid_for(count, BLOCK * 4);
    if (gb > 65536) gb = 65536;
    k_hub_owners<<<gb, BLOCK, 0, st>>>(verts, off, cpre, bpre, xpre, count, chunks, buckets);
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
// The moves of one workgroup's BLOCK vertices (positions t of the list),
// their community degree and size changes summed per community in LDS before
// the device atomics: a community that many movers enter or leave (a hub's)
// takes one update per workgroup instead of one per mover.  Called by the
// whole block; integer sums, so the result does not depend on the grouping.
constexpr int COMMIT_SLOTS = 4 * BLOCK; // two keys per mover: at most half full
struct CommitLds {
    int32_t key[COMMIT_SLOTS];
    long long da[COMMIT_SLOTS];
    int32_t dn[COMMIT_SLOTS];
};

__device__ __forceinline__ void commit_lds_add(CommitLds &L, int32_t c, long long da, int32_t dn)
{
    uint32_t slot = ((uint32_t)c * 2654435761u) & (COMMIT_SLOTS - 1);
    for (;;) {
        int32_t cur = L.key[slot];
        if (cur == -1) cur = atomicCAS(&L.key[slot], -1, c);
        if (cur == -1 || cur == c) {
            atomicAdd((unsigned long long *)&L.da[slot], (unsigned long long)da);
            atomicAdd(&L.dn[slot], dn);
            return;
        }
        slot = (slot + 1) & (COMMIT_SLOTS - 1);
    }
}

__device__ __forceinline__ void commit_tile(const int32_t *verts, int64_t t, int64_t count, int32_t *comm_prev,
                                            const int32_t *comm_next, const int64_t *k, int64_t *a, int32_t *size,
                                            CommitLds &L)
{
    static_assert((COMMIT_SLOTS & (COMMIT_SLOTS - 1)) == 0, "power-of-two table");
    for (int j = threadIdx.x; j < COMMIT_SLOTS; j += BLOCK) {
        L.key[j] = -1;
        L.da[j] = 0;
        L.dn[j] = 0;
    }
    __syncthreads();
    if (t < count) {
        const int32_t i = verts ? verts[t] : (int32_t)t;
        const int32_t A = comm_prev[i], B = comm_next[i];
        if (A != B) {
            const int64_t ki = k[i];
            commit_lds_add(L, A, -ki, -1);
            commit_lds_add(L, B, ki, 1);
            comm_prev[i] = B;
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < COMMIT_SLOTS; j += BLOCK) {
        const int32_t c = L.key[j];
        if (c < 0) continue;
        if (L.da[j]) atomicAdd((unsigned long long *)&a[c], (unsigned long long)L.da[j]);
        if (L.dn[j]) atomicAdd(&size[c], L.dn[j]);
    }
    __syncthreads(); // the table is cleared for the next tile
}

__global__ __launch_bounds__(BLOCK) void k_commit(const int32_t *verts, int64_t count, int32_t *comm_prev,
                                                  const int32_t *comm_next, const int64_t *k, int64_t *a,
                                                  int32_t *size)
{
    __shared__ CommitLds L;
    for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < count; base += (int64_t)gridDim.x * BLOCK)
        commit_tile(verts, base + threadIdx.x, count, comm_prev, comm_next, k, a, size, L);
}

void commit(const int32_t *verts, int64_t count, int32_t *comm_prev, const int32_t *comm_next, const int64_t *k,
            int64_t *a, int32_t *size, hipStream_t st)
{
    if (count <= 0) return;
    unsigned gc = grid_for(count, BLOCK);
    if (gc > 65536) gc = 65536;
    k_commit<<<gc, BLOCK, 0, st>>>(verts, count, comm_prev, comm_next, k, a, size);
}

// commit of a colour class: blocks [0, nb) commit the vertices before the
// class's hubs (positions [pos0, pos0 + count), hubs last in the class), the
// other blocks give one wavefront per hub, which decides and commits it
__device__ __forceinline__ void commit_one(int32_t i, int32_t B, int32_t *comm_prev, const int64_t *k, int64_t *ca,
                                           int32_t *size)
{
    const int32_t A = comm_prev[i];
    if (A == B) return;
    const int64_t ki = k[i];
    atomicAdd((unsigned long long *)&ca[A], (unsigned long long)(-ki));
    atomicAdd((unsigned long long *)&ca[B], (unsigned long long)ki);
    atomicSub(&size[A], 1);
    atomicAdd(&size[B], 1);
    comm_prev[i] = B;
}

template <typename GT>
__global__ __launch_bounds__(BLOCK) void k_commit_hubs(SweepArgs a, HubArgs h, const int32_t *list, int64_t pos0,
                                                       int64_t count, int64_t nplain, unsigned nb)
{
    int32_t *comm_prev = const_cast<int32_t *>(a.comm_prev);
    int64_t *ca = const_cast<int64_t *>(a.a);
    int32_t *size = const_cast<int32_t *>(a.size);
    if (blockIdx.x < nb) {
        __shared__ CommitLds L;
        for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < nplain; base += (int64_t)nb * BLOCK)
            commit_tile(list, base + threadIdx.x, nplain, comm_prev, a.comm_next, a.k, ca, size, L);
        return;
    }
    const int64_t nw = (int64_t)(gridDim.x - nb) * (BLOCK / 64);
    for (int64_t t = nplain + (int64_t)(blockIdx.x - nb) * (BLOCK / 64) + (threadIdx.x >> 6); t < count; t += nw) {
        const int32_t dest = hub_decide<GT>(a, h, pos0 + t);
        if ((threadIdx.x & 63) == 0) commit_one(list[t], dest, comm_prev, a.k, ca, size);
    }
}

void commit_hubs(const SweepArgs &a, const HubArgs &h, const int32_t *list, int64_t pos0, int64_t count, bool wide,
                 hipStream_t st)
{
    if (count <= 0) return;
    // the class's hubs are its last positions
    const int64_t nhub = (h.e > h.s) ? h.e - h.s : 0;
    const int64_t nplain = count - nhub;
    // one vertex per thread: a commit is a short chain of dependent reads
    // and atomics, and a class is small
    unsigned nb = grid_for(nplain > 0 ? nplain : 1, BLOCK);
    if (nb > 65536) nb = 65536;
    unsigned nh = nhub ? grid_for(nhub, BLOCK / 64) : 0;
    if (nh > 1024) nh = 1024;
    if (wide) k_commit_hubs<i128><<<nb + nh, BLOCK, 0, st>>>(a, h, list, pos0, count, nplain, nb);
    else k_commit_hubs<int64_t><<<nb + nh, BLOCK, 0, st>>>(a, h, list, pos0, count, nplain, nb);
}

void clear_stats(SweepStats *s, int count, hipStream_t st)
{
    fill<int64_t>((int64_t *)s, 0, (int64_t)count * (int64_t)(sizeof(SweepStats) / sizeof(int64_t)), st);
}

} // namespace lv
