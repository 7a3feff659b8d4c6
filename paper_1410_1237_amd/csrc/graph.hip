// Graph-level kernels: input validation, weighted degrees (Sec. 2), exact
// modularity pieces (Eq. 3), vertex following (Sec. 5.3) and the community
// graph rebuild between phases (Sec. 5.4 step 4) by radix sort of packed
// (C(u), C(v)) keys, run-length reduction and prefix-sum renumbering.
#include "lv.h"

namespace lv {

__device__ __forceinline__ int64_t wave_sum(int64_t v)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        int lo = __shfl_xor((int)(uint32_t)v, d, 64);
        int hi = __shfl_xor((int)(v >> 32), d, 64);
        v += (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    }
    return v;
}

__device__ __forceinline__ int64_t block_total(int64_t v, int64_t *s)
{
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t t = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) t += s[w];
    __syncthreads();
    return t;
}

// ---- validation ---------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_validate_offsets(const int64_t *off, int64_t n, int64_t nnz, int32_t *flag)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        if (off[i + 1] < off[i]) atomicCAS(flag, 0, 1);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        if (off[0] != 0 || off[n] != nnz) atomicCAS(flag, 0, 1);
}

template <int WK>
__global__ __launch_bounds__(BLOCK) void k_validate_entries(Csr g, int full, int32_t *flag)
{
    __shared__ int64_t s_off[ROWCAP + 1];
    __shared__ int64_t s_meta[2];
    const int64_t e0 = (int64_t)blockIdx.x * ETILE;
    const int64_t e1 = min(e0 + ETILE, g.nnz) - 1;
    TileRows t = tile_rows(g.off, g.n, e0, e1, s_off, s_meta);
    for (int r = 0; r < EITEMS; ++r) {
        const int64_t e = e0 + r * BLOCK + threadIdx.x;
        if (e > e1) break;
        const int64_t u = tile_row(t, g.off, s_off, e);
        const int32_t v = g.col[e];
        const int64_t w = WLoad<WK>::at(g.w, e);
        if (v < 0 || v >= g.n) { atomicCAS(flag, 0, 2); continue; }
        if (!full) continue;
        if (e > tile_off(t, g.off, s_off, u) && g.col[e - 1] >= v) atomicCAS(flag, 0, 3);
        if (w < 1) atomicCAS(flag, 0, 4);
        // mirror (v, u) with the same weight: binary search in row v
        int64_t lo = g.off[v], hi = g.off[v + 1];
        bool ok = false;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            int32_t c = g.col[mid];
            if (c == u) { ok = WLoad<WK>::at(g.w, mid) == w; break; }
            if (c < u) lo = mid + 1; else hi = mid;
        }
        if (!ok) atomicCAS(flag, 0, 5);
    }
}

void validate_csr(const Csr &g, int32_t *flag, hipStream_t st)
{
    fill<int32_t>(flag, 0, 1, st);
    unsigned gv = grid_for(g.n, BLOCK * 8);
    if (gv > 65536) gv = 65536;
    k_validate_offsets<<<gv, BLOCK, 0, st>>>(g.off, g.n, g.nnz, flag);
}

void validate_entries(const Csr &g, bool full, int32_t *flag, hipStream_t st)
{
    if (g.nnz == 0) return;
    unsigned ge = grid_for(g.nnz, ETILE);
    switch (g.wk) {
    case W_UNIT: k_validate_entries<W_UNIT><<<ge, BLOCK, 0, st>>>(g, full, flag); break;
    case W_I32: k_validate_entries<W_I32><<<ge, BLOCK, 0, st>>>(g, full, flag); break;
    default: k_validate_entries<W_I64><<<ge, BLOCK, 0, st>>>(g, full, flag); break;
    }
}

// ---- degrees -----------------------------------------------------------------
// Each thread sums EITEMS consecutive entries per row; partial row sums are
// combined in LDS when the tile's rows are cached (one global atomic per row
// and block), else added to k directly.
template <int WK>
__global__ __launch_bounds__(BLOCK) void k_degrees(Csr g, int64_t *k, int64_t *rep, int32_t *range_flag)
{
    __shared__ int64_t s_off[ROWCAP + 1];
    __shared__ int64_t s_meta[2];
    __shared__ int64_t s_red[BLOCK / 64];
    __shared__ unsigned long long s_acc[ROWCAP + 1];
    const int64_t e0 = (int64_t)blockIdx.x * ETILE;
    const int64_t e1 = min(e0 + ETILE, g.nnz) - 1;
    TileRows t = tile_rows(g.off, g.n, e0, e1, s_off, s_meta);
    const int64_t nrows = t.rhi - t.rlo + 1;
    if (t.cached)
        for (int64_t j = threadIdx.x; j < nrows; j += BLOCK) s_acc[j] = 0;
    __syncthreads();
    const int64_t b = e0 + (int64_t)threadIdx.x * EITEMS;
    const int64_t e_end = min(b + EITEMS, e1 + 1);
    int64_t tot = 0, self = 0;
    if (b <= e1) {
        int64_t row = tile_row(t, g.off, s_off, b);
        int64_t next = tile_off(t, g.off, s_off, row + 1);
        int64_t acc = 0;
        for (int64_t e = b; e < e_end; ++e) {
            while (e >= next) {
                if (acc) {
                    if (t.cached) atomicAdd(&s_acc[row - t.rlo], (unsigned long long)acc);
                    else atomicAdd((unsigned long long *)&k[row], (unsigned long long)acc);
                }
                acc = 0;
                ++row;
                next = tile_off(t, g.off, s_off, row + 1);
                if (e >= next) { // empty rows: search instead of stepping through them
                    row = tile_row(t, g.off, s_off, e);
                    next = tile_off(t, g.off, s_off, row + 1);
                }
            }
            const int64_t w = WLoad<WK>::at(g.w, e);
            const int32_t c = g.col[e];
            acc += w;
            tot += w;
            if (c == row) self += w;
            if (range_flag && (c < 0 || c >= g.n)) atomicCAS(range_flag, 0, 2); // the column check, same pass
        }
        if (acc) {
            if (t.cached) atomicAdd(&s_acc[row - t.rlo], (unsigned long long)acc);
            else atomicAdd((unsigned long long *)&k[row], (unsigned long long)acc);
        }
    }
    __syncthreads();
    if (t.cached)
        for (int64_t j = threadIdx.x; j < nrows; j += BLOCK)
            if (s_acc[j]) atomicAdd((unsigned long long *)&k[t.rlo + j], s_acc[j]);
    tot = block_total(tot, s_red);
    self = block_total(self, s_red);
    if (threadIdx.x == 0) {
        rep_add(rep, 0, tot);
        rep_add(rep, 2, self);
    }
}

// flag = 2 if a column lies outside [0, n)
__global__ __launch_bounds__(BLOCK) void k_col_range(const int32_t *col, int64_t nnz, int64_t n, int32_t *flag)
{
    bool bad = false;
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * BLOCK) {
        const int32_t c = col[e];
        bad |= c < 0 || c >= n;
    }
    if (bad) atomicCAS(flag, 0, 2);
}

// unit weights: k_v is the row length, and the columns of
// a row are strictly ascending, so its self-loop is found by a binary search
// of the row for v (a thread per row; 2m and the self-loop count into the
// replicated counters 0 and 2).  No column is used as an index, so this is
// safe before the column check has run.
__global__ __launch_bounds__(BLOCK) void k_degrees_unit(Csr g, int64_t *k, int64_t *rep)
{
    __shared__ int64_t s_red[BLOCK / 64];
    int64_t tot = 0, self = 0;
    for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < g.n; v += (int64_t)gridDim.x * BLOCK) {
        int64_t lo = g.off[v], hi = g.off[v + 1];
        k[v] = hi - lo;
        tot += hi - lo;
        while (lo < hi) { // first column >= v
            const int64_t mid = (lo + hi) >> 1;
            if (g.col[mid] < v) lo = mid + 1;
            else hi = mid;
        }
        if (lo < g.off[v + 1] && g.col[lo] == v) ++self;
    }
    tot = block_total(tot, s_red);
    self = block_total(self, s_red);
    if (threadIdx.x == 0) {
        rep_add(rep, 0, tot);
        rep_add(rep, 2, self);
    }
}

__global__ __launch_bounds__(BLOCK) void k_max(const int64_t *k, int64_t n, int64_t *out)
{
    __shared__ int64_t s[BLOCK / 64];
    int64_t m = 0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        m = max(m, k[i]);
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        int lo = __shfl_xor((int)(uint32_t)m, d, 64);
        int hi = __shfl_xor((int)(m >> 32), d, 64);
        m = max(m, (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
    }
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int w = 0; w < BLOCK / 64; ++w) t = max(t, s[w]);
        atomicMax((unsigned long long *)out, (unsigned long long)t);
    }
}

constexpr int REP_FOLD_THREADS = 64 * 8; // one wave per counter, one lane per replica

__global__ __launch_bounds__(REP_FOLD_THREADS) void k_rep_fold(const int64_t *rep, int count, int64_t *out)
{
    const int c = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (c >= count) return;
    int64_t v = rep[8 * lane + c];
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        int lo = __shfl_xor((int)(uint32_t)v, d, 64);
        int hi = __shfl_xor((int)(v >> 32), d, 64);
        v += (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    }
    if (lane == 0) out[c] = v;
}

void rep_clear(int64_t *rep, hipStream_t st) { fill<int64_t>(rep, 0, 8 * RED_REP, st); }

void rep_fold(const int64_t *rep, int count, int64_t *out, hipStream_t st)
{
    static_assert(RED_REP == 64, "one lane per replica");
    k_rep_fold<<<1, REP_FOLD_THREADS, 0, st>>>(rep, count, out);
}

void degrees(const Csr &g, int64_t *k, int64_t *stats, Scratch &s, hipStream_t st, int32_t *range_flag)
{
    fill<int64_t>(k, 0, g.n, st);
    fill<int64_t>(stats, 0, 3, st);
    rep_clear(s.rep, st);
    if (g.nnz > 0 && g.wk == W_UNIT) {
        if (range_flag) { // the column check, a stream over the columns
            unsigned gc = grid_for(g.nnz, BLOCK * 16);
            if (gc > 65536) gc = 65536;
            k_col_range<<<gc, BLOCK, 0, st>>>(g.col, g.nnz, g.n, range_flag);
        }
        unsigned gn = grid_for(g.n, BLOCK * 4);
        if (gn > 65536) gn = 65536;
        k_degrees_unit<<<gn, BLOCK, 0, st>>>(g, k, s.rep);
    } else if (g.nnz > 0) {
        unsigned ge = grid_for(g.nnz, ETILE);
        switch (g.wk) {
        case W_UNIT: k_degrees<W_UNIT><<<ge, BLOCK, 0, st>>>(g, k, s.rep, range_flag); break;
        case W_I32: k_degrees<W_I32><<<ge, BLOCK, 0, st>>>(g, k, s.rep, range_flag); break;
        default: k_degrees<W_I64><<<ge, BLOCK, 0, st>>>(g, k, s.rep, range_flag); break;
        }
    }
    rep_fold(s.rep, 3, stats, st); // 2m, 0 (the maximum comes next), self-loops
    if (g.n > 0) {
        unsigned gm = grid_for(g.n, BLOCK * 16);
        if (gm > 4096) gm = 4096;
        k_max<<<gm, BLOCK, 0, st>>>(k, g.n, stats + 1);
    }
}

// ---- sum of squares (128-bit) ------------------------------------------------
constexpr int SQ_GRID = 1024;

__global__ __launch_bounds__(BLOCK) void k_sumsq(const int64_t *a, int64_t n, u128 *part)
{
    __shared__ u128 s[BLOCK];
    u128 acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        const int64_t x = a[i];
        acc += (u128)((i128)x * x);
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = BLOCK / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(BLOCK) void k_sumsq_final(const u128 *part, int nparts, int64_t *out)
{
    __shared__ u128 s[BLOCK];
    u128 acc = 0;
    for (int i = threadIdx.x; i < nparts; i += BLOCK) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = BLOCK / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = (int64_t)(uint64_t)s[0];
        out[1] = (int64_t)(uint64_t)(s[0] >> 64);
    }
}

void sum_squares(const int64_t *a, int64_t n, int64_t *out, Scratch &s, hipStream_t st)
{
    u128 *part = (u128 *)s.part;
    unsigned gq = grid_for(n, BLOCK * 4);
    if (gq > SQ_GRID) gq = SQ_GRID;
    k_sumsq<<<gq, BLOCK, 0, st>>>(a, n, part);
    k_sumsq_final<<<1, BLOCK, 0, st>>>(part, (int)gq, out);
}

// ---- internal weight of a partition -----------------------------------------
template <int WK>
__global__ __launch_bounds__(BLOCK) void k_internal(Csr g, const int32_t *comm, int64_t *rep)
{
    __shared__ int64_t s_off[ROWCAP + 1];
    __shared__ int64_t s_meta[2];
    __shared__ int64_t s_red[BLOCK / 64];
    const int64_t e0 = (int64_t)blockIdx.x * ETILE;
    const int64_t e1 = min(e0 + ETILE, g.nnz) - 1;
    TileRows t = tile_rows(g.off, g.n, e0, e1, s_off, s_meta);
    int64_t acc = 0;
    for (int r = 0; r < EITEMS; ++r) {
        const int64_t e = e0 + r * BLOCK + threadIdx.x;
        if (e > e1) break;
        const int64_t u = tile_row(t, g.off, s_off, e);
        if (comm[u] == comm[g.col[e]]) acc += WLoad<WK>::at(g.w, e);
    }
    acc = block_total(acc, s_red);
    if (threadIdx.x == 0) rep_add(rep, 0, acc);
}

void internal_weight(const Csr &g, const int32_t *comm, int64_t *out, Scratch &s, hipStream_t st)
{
    rep_clear(s.rep, st);
    if (g.nnz > 0) {
        unsigned ge = grid_for(g.nnz, ETILE);
        switch (g.wk) {
        case W_UNIT: k_internal<W_UNIT><<<ge, BLOCK, 0, st>>>(g, comm, s.rep); break;
        case W_I32: k_internal<W_I32><<<ge, BLOCK, 0, st>>>(g, comm, s.rep); break;
        default: k_internal<W_I64><<<ge, BLOCK, 0, st>>>(g, comm, s.rep); break;
        }
    }
    rep_fold(s.rep, 1, out, st);
}

// ---- vertex following -----------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_vf(const int64_t *off, const int32_t *col, int64_t n, int32_t *map)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        int32_t m = (int32_t)i;
        const int64_t b = off[i];
        if (off[i + 1] - b == 1 && col[b] != i) {
            const int32_t j = col[b];
            const bool j_single = (off[j + 1] - off[j] == 1); // its one entry is (j, i)
            m = j_single ? min((int32_t)i, j) : j;
        }
        map[i] = m;
    }
}

void vf_map(const Csr &g, int32_t *map, hipStream_t st)
{
    if (g.n == 0) return;
    unsigned gv = grid_for(g.n, BLOCK * 4);
    if (gv > 65536) gv = 65536;
    k_vf<<<gv, BLOCK, 0, st>>>(g.off, g.col, g.n, map);
}

// the one neighbour j != i of row i and its weight, if the row holds exactly
// one besides an optional self-loop (rows are sorted and have no repeats, so
// such a row has one or two entries)
template <int WK>
__device__ __forceinline__ bool one_neighbour(const Csr &g, int64_t i, int32_t &j, int64_t &w)
{
    const int64_t b = g.off[i], len = g.off[i + 1] - b;
    if (len == 1) {
        j = g.col[b];
        w = WLoad<WK>::at(g.w, b);
        return j != i;
    }
    if (len == 2) {
        const int32_t c0 = g.col[b], c1 = g.col[b + 1];
        if (c0 == i || c1 == i) {
            const int64_t e = c0 == i ? b + 1 : b;
            j = g.col[e];
            w = WLoad<WK>::at(g.w, e);
            return true;
        }
    }
    return false;
}

// one round of chain-compressing vertex following (the extension closing
// Sec. 5.3): i qualifies when it has a single neighbour j and the bound of
// Lemma 3's proof is positive, 2m * w_ij > k_i * k_j (the gain of moving i
// into j's one-vertex community, Eq. 4, exact in 128 bits); it then follows j,
// or the smaller id of the two when j qualifies as well (they only see each
// other).  2m is the graph's own (g_two_m[gid[i]] in a batch).  Counter 0 of
// rep gets the vertices that follow another.
template <int WK>
__global__ __launch_bounds__(BLOCK) void k_vf_chain(Csr g, const int64_t *k, int64_t two_m, const int32_t *gid,
                                                    const int64_t *g_two_m, int32_t *map, int64_t *rep)
{
    __shared__ int64_t s_red[BLOCK / 64];
    int64_t moved = 0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < g.n; i += (int64_t)gridDim.x * BLOCK) {
        int32_t m = (int32_t)i, j, jj;
        int64_t w, wj;
        const int64_t tm = gid ? g_two_m[gid[i]] : two_m;
        if (one_neighbour<WK>(g, i, j, w) && (__int128)tm * w > (__int128)k[i] * k[j]) {
            m = j;
            if (one_neighbour<WK>(g, j, jj, wj) && (__int128)tm * wj > (__int128)k[j] * k[i]) m = min((int32_t)i, j);
        }
        map[i] = m;
        moved += m != i;
    }
    moved = block_total(moved, s_red);
    if (threadIdx.x == 0) rep_add(rep, 0, moved);
}

void vf_chain_map(const Csr &g, const int64_t *k, int64_t two_m, const int32_t *gid, const int64_t *g_two_m,
                  int32_t *map, int64_t *moved, Scratch &s, hipStream_t st)
{
    rep_clear(s.rep, st);
    if (g.n > 0) {
        unsigned gv = grid_for(g.n, BLOCK * 4);
        if (gv > 65536) gv = 65536;
        switch (g.wk) {
        case W_UNIT: k_vf_chain<W_UNIT><<<gv, BLOCK, 0, st>>>(g, k, two_m, gid, g_two_m, map, s.rep); break;
        case W_I32: k_vf_chain<W_I32><<<gv, BLOCK, 0, st>>>(g, k, two_m, gid, g_two_m, map, s.rep); break;
        default: k_vf_chain<W_I64><<<gv, BLOCK, 0, st>>>(g, k, two_m, gid, g_two_m, map, s.rep); break;
        }
    }
    rep_fold(s.rep, 1, moved, st);
}

// ---- coarsening ---------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_mark(const int32_t *comm, int64_t n, int32_t *flag)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        flag[comm[i]] = 1;
}

__global__ __launch_bounds__(BLOCK) void k_compose(int32_t *orig_map, int64_t n_orig, const int32_t *comm,
                                                   const int32_t *new_id)
{
    for (int64_t x = (int64_t)blockIdx.x * BLOCK + threadIdx.x; x < n_orig; x += (int64_t)gridDim.x * BLOCK)
        orig_map[x] = new_id[comm[orig_map[x]]];
}

// cmap[v] = new id of the community of v
__global__ __launch_bounds__(BLOCK) void k_cmap(const int32_t *comm, const int32_t *new_id, int64_t n, int32_t *cmap)
{
    for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * BLOCK)
        cmap[v] = new_id[comm[v]];
}

// The rebuild's keys, one per CSR entry (the sort's input when the tile sums
// below would not shrink it: keys only for unit weights, whose run lengths
// are the weights)
template <int WK, bool HV>
__global__ __launch_bounds__(BLOCK) void k_coarse_keys(Csr g, const int32_t *cmap, int bits, uint64_t *keys,
                                                       int64_t *vals)
{
    __shared__ int64_t s_off[ROWCAP + 1];
    __shared__ int64_t s_meta[2];
    const int64_t e0 = (int64_t)blockIdx.x * ETILE;
    const int64_t e1 = min(e0 + ETILE, g.nnz) - 1;
    TileRows t = tile_rows(g.off, g.n, e0, e1, s_off, s_meta);
    for (int r = 0; r < EITEMS; ++r) {
        const int64_t e = e0 + r * BLOCK + threadIdx.x;
        if (e > e1) break;
        const int64_t u = tile_row(t, g.off, s_off, e);
        const uint64_t cu = (uint32_t)cmap[u];
        const uint64_t cv = (uint32_t)cmap[g.col[e]];
        keys[e] = (cu << bits) | cv;
        if (HV) vals[e] = WLoad<WK>::at(g.w, e);
    }
}

// The rebuild's (C(u) << bits | C(v), w) pairs, summed per key inside each
// tile of PAIR_TILE consecutive entries before the sort: after a phase most
// neighbours of a row (and of the rows around it) fall into a few
// communities, so a tile holds far fewer distinct keys than entries (about a
// sixth on R-MAT after its first phase), and the radix sort and everything
// after it run over the tile sums.  Equal keys of different tiles stay
// separate here and are summed with the runs after the sort (integer sums,
// so the coarse graph does not depend on the order in which tiles append).
// Each tile sums in an LDS table with twice as many slots as entries (linear
// probing, ~0 marks a free slot: keys are below 2^62), then appends its
// distinct keys behind an atomic counter.
constexpr int PAIR_ITEMS = 4;
constexpr int PAIR_TILE = BLOCK * PAIR_ITEMS;
constexpr int PAIR_SLOTS = 2 * PAIR_TILE;
constexpr int PAIR_SHIFT = 64 - 11; // log2(PAIR_SLOTS) = 11
static_assert(PAIR_SLOTS == 1 << 11, "table index bits");
constexpr uint64_t PAIR_FREE = ~0ull;

template <int WK>
__global__ __launch_bounds__(BLOCK) void k_coarse_pairs(Csr g, const int32_t *cmap, int bits, uint64_t *keys,
                                                        int64_t *vals, unsigned long long *count)
{
    __shared__ int64_t s_off[ROWCAP + 1];
    __shared__ int64_t s_meta[2];
    __shared__ uint64_t s_key[PAIR_SLOTS];
    __shared__ int64_t s_w[PAIR_SLOTS];
    __shared__ int32_t s_wsum[BLOCK / 64];
    __shared__ unsigned long long s_base;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int j = tid; j < PAIR_SLOTS; j += BLOCK) {
        s_key[j] = PAIR_FREE;
        s_w[j] = 0;
    }
    const int64_t e0 = (int64_t)blockIdx.x * PAIR_TILE;
    const int64_t e1 = min(e0 + PAIR_TILE, g.nnz) - 1;
    TileRows t = tile_rows(g.off, g.n, e0, e1, s_off, s_meta); // ends with a block barrier
    // the tile's keys, every gather issued before any insertion
    uint64_t key[PAIR_ITEMS];
    int64_t w[PAIR_ITEMS];
#pragma unroll
    for (int r = 0; r < PAIR_ITEMS; ++r) {
        const int64_t e = e0 + r * BLOCK + tid;
        key[r] = PAIR_FREE;
        w[r] = 0;
        if (e <= e1) {
            const int64_t u = tile_row(t, g.off, s_off, e);
            key[r] = ((uint64_t)(uint32_t)cmap[u] << bits) | (uint64_t)(uint32_t)cmap[g.col[e]];
            w[r] = WLoad<WK>::at(g.w, e);
        }
    }
#pragma unroll
    for (int r = 0; r < PAIR_ITEMS; ++r) {
        if (key[r] == PAIR_FREE) continue;
        uint32_t slot = (uint32_t)((key[r] * 0x9E3779B97F4A7C15ull) >> PAIR_SHIFT);
        for (;;) {
            uint64_t cur = s_key[slot];
            if (cur == PAIR_FREE) cur = atomicCAS((unsigned long long *)&s_key[slot], PAIR_FREE, key[r]);
            if (cur == PAIR_FREE || cur == key[r]) {
                atomicAdd((unsigned long long *)&s_w[slot], (unsigned long long)w[r]);
                break;
            }
            slot = (slot + 1) & (PAIR_SLOTS - 1);
        }
    }
    __syncthreads();
    // append: thread tid owns the slots [tid * SPT, (tid + 1) * SPT)
    constexpr int SPT = PAIR_SLOTS / BLOCK;
    int32_t c = 0;
#pragma unroll
    for (int i = 0; i < SPT; ++i) c += s_key[tid * SPT + i] != PAIR_FREE;
    int32_t inc = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) s_wsum[wid] = inc;
    __syncthreads();
    int32_t pre = inc - c, total = 0;
#pragma unroll
    for (int v = 0; v < BLOCK / 64; ++v) {
        if (v < wid) pre += s_wsum[v];
        total += s_wsum[v];
    }
    if (tid == 0) s_base = atomicAdd(count, (unsigned long long)total);
    __syncthreads();
    int64_t pos = (int64_t)s_base + pre;
#pragma unroll
    for (int i = 0; i < SPT; ++i) {
        const uint64_t k = s_key[tid * SPT + i];
        if (k == PAIR_FREE) continue;
        keys[pos] = k;
        vals[pos] = s_w[tid * SPT + i];
        ++pos;
    }
}

// heads of sorted key runs: run r starts at rstart[r]; column and row of r
__global__ __launch_bounds__(BLOCK) void k_runs(const uint64_t *keys, const int64_t *run, int64_t nnz, int bits,
                                                int64_t *rstart, int32_t *col_out)
{
    const uint64_t mask = (bits >= 64) ? ~0ull : ((1ull << bits) - 1);
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * BLOCK) {
        if (e == 0 || keys[e] != keys[e - 1]) {
            const int64_t r = run[e];
            rstart[r] = e;
            col_out[r] = (int32_t)(keys[e] & mask);
        }
    }
}

// weight of every run (summed entries of one (C(u), C(v)) pair); the
// diagonal runs (self-loops of the coarse graph) are also summed into rep
__global__ __launch_bounds__(BLOCK) void k_run_weights(const uint64_t *keys, int bits, const int64_t *rstart,
                                                       int64_t nruns, const int64_t *pref, int64_t *w_out,
                                                       int64_t *rep)
{
    __shared__ int64_t s_red[BLOCK / 64];
    const uint64_t mask = (bits >= 64) ? ~0ull : ((1ull << bits) - 1);
    int64_t diag = 0;
    for (int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x; r < nruns; r += (int64_t)gridDim.x * BLOCK) {
        const int64_t w = pref ? pref[rstart[r + 1]] - pref[rstart[r]] : rstart[r + 1] - rstart[r];
        w_out[r] = w;
        const uint64_t key = keys[rstart[r]];
        if ((key >> bits) == (key & mask)) diag += w;
    }
    diag = block_total(diag, s_red);
    if (threadIdx.x == 0) rep_add(rep, 0, diag);
}

// weighted degrees of the coarse graph: the sum of the sorted entries of row c
__global__ __launch_bounds__(BLOCK) void k_coarse_degrees(const int64_t *off, const int64_t *rstart, const int64_t *pref,
                                                          int64_t n, int64_t *k)
{
    for (int64_t c = (int64_t)blockIdx.x * BLOCK + threadIdx.x; c < n; c += (int64_t)gridDim.x * BLOCK) {
        const int64_t lo = rstart[off[c]], hi = rstart[off[c + 1]];
        k[c] = pref ? pref[hi] - pref[lo] : hi - lo;
    }
}

// runs per coarse row, counted from the first and the last run of each row
// (at most two uncontended additions per row; rows with no run stay 0); an
// exclusive scan then gives the row offsets. Work per thread is one run,
// whatever the lengths of the rows or of the gaps between non-empty rows.
__global__ __launch_bounds__(BLOCK) void k_row_counts(const uint64_t *keys, const int64_t *rstart, int64_t nruns,
                                                      int bits, int64_t *cnt)
{
    for (int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x; r < nruns; r += (int64_t)gridDim.x * BLOCK) {
        const uint64_t row = keys[rstart[r]] >> bits;
        const bool head = r == 0 || (keys[rstart[r - 1]] >> bits) != row;
        const bool tail = r == nruns - 1 || (keys[rstart[r + 1]] >> bits) != row;
        unsigned long long *c = (unsigned long long *)&cnt[row];
        if (head && tail) *c = 1;
        else if (head) atomicAdd(c, (unsigned long long)(-r));
        else if (tail) atomicAdd(c, (unsigned long long)(r + 1));
    }
}

static int bits_for(int64_t n)
{
    int b = 1;
    while (((int64_t)1 << b) < n) ++b;
    return b;
}

hipError_t coarsen(const Csr &g, const int32_t *comm, int32_t *orig_map, int64_t n_orig, CoarsenBufs &b,
                   int64_t *off_out, int32_t *col_out, int64_t *w_out, int64_t *k_out, int64_t *stats, int64_t *n_new,
                   int64_t *nnz_new, Scratch &s, hipStream_t st, bool tile_sums)
{
    fill<int64_t>(stats, 0, 3, st);
    const int64_t n = g.n, nnz = g.nnz;
    // renumber non-empty communities in ascending id
    fill<int32_t>(b.flag, 0, n + 1, st);
    unsigned gv = grid_for(n, BLOCK * 4);
    if (gv > 65536) gv = 65536;
    if (n > 0) k_mark<<<gv, BLOCK, 0, st>>>(comm, n, b.flag);
    scan_i32_to_i32(b.flag, b.new_id, n, s.scalar, s, st);
    int64_t nn = 0;
    if (const hipError_t e = read_back(&nn, s.scalar, st)) return e;
    unsigned gx = grid_for(n_orig, BLOCK * 4);
    if (gx > 65536) gx = 65536;
    if (n_orig > 0) k_compose<<<gx, BLOCK, 0, st>>>(orig_map, n_orig, comm, b.new_id);
    *n_new = nn;
    if (nnz == 0) {
        fill<int64_t>(off_out, 0, nn + 1, st);
        fill<int64_t>(k_out, 0, nn, st);
        *nnz_new = 0;
        return hipGetLastError();
    }
    const int bits = bits_for(nn > 1 ? nn : 2);
    int32_t *cmap = b.flag; // free after the renumbering scan
    k_cmap<<<gv, BLOCK, 0, st>>>(comm, b.new_id, n, cmap);
    // the sort's np (key, weight) pairs: tile sums, or one per entry (keys
    // only for unit weights: hv false, weights are run lengths)
    int64_t np = nnz;
    bool hv = true;
    if (tile_sums) {
        fill<int64_t>(s.scalar, 0, 1, st);
        const unsigned gp = grid_for(nnz, PAIR_TILE);
        unsigned long long *cnt = (unsigned long long *)s.scalar;
        switch (g.wk) {
        case W_UNIT: k_coarse_pairs<W_UNIT><<<gp, BLOCK, 0, st>>>(g, cmap, bits, b.keys, b.vals, cnt); break;
        case W_I32: k_coarse_pairs<W_I32><<<gp, BLOCK, 0, st>>>(g, cmap, bits, b.keys, b.vals, cnt); break;
        default: k_coarse_pairs<W_I64><<<gp, BLOCK, 0, st>>>(g, cmap, bits, b.keys, b.vals, cnt); break;
        }
        if (const hipError_t e = read_back(&np, s.scalar, st)) return e;
    } else {
        hv = g.wk != W_UNIT;
        const unsigned ge = grid_for(nnz, ETILE);
        switch (g.wk) {
        case W_UNIT: k_coarse_keys<W_UNIT, false><<<ge, BLOCK, 0, st>>>(g, cmap, bits, b.keys, nullptr); break;
        case W_I32: k_coarse_keys<W_I32, true><<<ge, BLOCK, 0, st>>>(g, cmap, bits, b.keys, b.vals); break;
        default: k_coarse_keys<W_I64, true><<<ge, BLOCK, 0, st>>>(g, cmap, bits, b.keys, b.vals); break;
        }
    }
    radix_sort(b.keys, b.keys_alt, hv ? b.vals : nullptr, b.vals_alt, np, 2 * bits, s, st);
    scan_heads(b.keys, b.run, np, s.scalar, s, st);
    int64_t nruns = 0;
    if (const hipError_t e = read_back(&nruns, s.scalar, st)) return e;
    int64_t *rstart = b.vals_alt; // free after the sort; np + 1 entries
    unsigned gr = grid_for(np, BLOCK * 4);
    if (gr > 65536) gr = 65536;
    k_runs<<<gr, BLOCK, 0, st>>>(b.keys, b.run, np, bits, rstart, col_out);
    fill<int64_t>(rstart + nruns, np, 1, st);
    int64_t *pref = nullptr;
    if (hv) {
        pref = (int64_t *)b.keys_alt; // exclusive prefix of the sorted weights, np + 1 entries
        scan_i64(b.vals, pref, np, pref + np, s, st);
    }
    unsigned gw = grid_for(nruns, BLOCK * 4);
    if (gw > 65536) gw = 65536;
    rep_clear(s.rep, st);
    k_run_weights<<<gw, BLOCK, 0, st>>>(b.keys, bits, rstart, nruns, pref, w_out, s.rep);
    fill<int64_t>(off_out, 0, nn, st);
    k_row_counts<<<gw, BLOCK, 0, st>>>(b.keys, rstart, nruns, bits, off_out);
    scan_i64(off_out, off_out, nn, off_out + nn, s, st); // in place; the total is nruns
    *nnz_new = nruns;
    // weighted degrees, 2m (the total weight: unchanged by coarsening), the
    // largest degree and the self-loop total of the coarse graph
    if (nn > 0) {
        unsigned gk = grid_for(nn, BLOCK * 4);
        if (gk > 65536) gk = 65536;
        k_coarse_degrees<<<gk, BLOCK, 0, st>>>(off_out, rstart, pref, nn, k_out);
        unsigned gm = grid_for(nn, BLOCK * 16);
        if (gm > 4096) gm = 4096;
        k_max<<<gm, BLOCK, 0, st>>>(k_out, nn, stats + 1);
    }
    if (pref) {
        if (const hipError_t e = hipMemcpyAsync(stats, pref + np, sizeof(int64_t), hipMemcpyDeviceToDevice, st))
            return e;
    } else {
        fill<int64_t>(stats, np, 1, st);
    }
    rep_fold(s.rep, 1, stats + 2, st);
    return hipGetLastError();
}

// ---- rebuild after vertex following -------------------------------------------
// Under a vertex-following map each community is one kept vertex u (a fixed
// point of the map) with the vertices whose only neighbour is u, so the
// coarse row of u is u's row without the entries into its own community,
// columns renumbered (the renumbering is monotone on the kept vertices, so
// the row stays sorted), plus the self-loop that collects everything inside
// the community: w_uu and the absorbed vertices' self-loops once, every edge
// to an absorbed vertex twice (both of its directions lie inside).  Entry
// tags in A: >= 0 the coarse column, else one of the following.
constexpr int32_t VF_INSIDE = -1; // entry to a vertex the row's vertex absorbs
constexpr int32_t VF_DROP = -2;   // entry of an absorbed vertex's row
constexpr int32_t VF_SELF = -3;   // the row's own self-loop

// wself[u]: u's own self-loop; aself[u]: the absorbed vertices' self-loops
// (zero unless a chain round absorbs vertices that carry one)
// kept-vertex bitmap of a vertex-following map: bit v & 63 of word v >> 6
// is set for a kept vertex, and kpre[w] counts the kept vertices before word
// w, so a kept vertex's new id is kpre[v >> 6] + the set bits below it; the
// two arrays (12 bytes per 64 vertices) stay in L2 where cmap (4 bytes per
// vertex) would be a line fetch per entry.  One wavefront per word.
__global__ __launch_bounds__(BLOCK) void k_keep_bits(const int32_t *flag, const int32_t *new_id, int64_t n,
                                                     uint64_t *kbits, int32_t *kpre)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = (n + 63) / 64;
    for (int64_t w = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) >> 6; w < nw;
         w += ((int64_t)gridDim.x * BLOCK) >> 6) {
        const int64_t v = w * 64 + lane;
        const uint64_t m = __ballot(v < n && flag[v] != 0);
        if (lane == 0) {
            kbits[w] = m;
            kpre[w] = new_id[w * 64];
        }
    }
}

template <int WK>
__global__ __launch_bounds__(BLOCK) void k_vf_entries(Csr g, const int32_t *map, const int32_t *cmap,
                                                      const uint64_t *kbits, const int32_t *kpre, int32_t *A,
                                                      int64_t *wself, int64_t *aself)
{
    __shared__ int64_t s_off[ROWCAP + 1];
    __shared__ int64_t s_meta[2];
    const int64_t e0 = (int64_t)blockIdx.x * ETILE;
    const int64_t e1 = min(e0 + ETILE, g.nnz) - 1;
    TileRows t = tile_rows(g.off, g.n, e0, e1, s_off, s_meta);
    for (int r = 0; r < EITEMS; ++r) {
        const int64_t e = e0 + r * BLOCK + threadIdx.x;
        if (e > e1) break;
        const int64_t u = tile_row(t, g.off, s_off, e);
        const int32_t v = g.col[e];
        if (map[u] != u) {
            A[e] = VF_DROP;
            if (v == u)
                atomicAdd((unsigned long long *)&aself[map[u]], (unsigned long long)WLoad<WK>::at(g.w, e));
            continue;
        }
        if (v == u) {
            A[e] = VF_SELF;
            wself[u] = WLoad<WK>::at(g.w, e);
            continue;
        }
        // the neighbour's new id: from the kept-vertex bitmap when it is kept,
        // else (an absorbed vertex) from the map
        int32_t cv;
        if (kbits) {
            const uint64_t word = kbits[v >> 6];
            cv = ((word >> (v & 63)) & 1) ? kpre[v >> 6] + __popcll(word & ((1ull << (v & 63)) - 1)) : cmap[v];
        } else {
            cv = cmap[v];
        }
        A[e] = cv == cmap[u] ? VF_INSIDE : cv;
    }
}

// entries of each coarse row (turned into offsets by a scan) and the
// community degree k_u + the weight of u's edges to the vertices it absorbs +
// their self-loops (the absorbed degrees); run / pin: exclusive prefix counts
// of the kept entries and prefix sums of the inside entries' weights, nnz + 1
// entries each.  kt holds the absorbed self-loops (aself) on entry; wself[u]
// becomes everything but the inside edges of the community's self-loop.
__global__ __launch_bounds__(BLOCK) void k_vf_rows(const int64_t *off, int64_t n, const int32_t *map,
                                                   const int32_t *cmap, const int64_t *run, const int64_t *pin,
                                                   int64_t *wself, const int64_t *k_in, int64_t *cnt_out,
                                                   int64_t *kt)
{
    for (int64_t u = (int64_t)blockIdx.x * BLOCK + threadIdx.x; u < n; u += (int64_t)gridDim.x * BLOCK) {
        if (map[u] != u) continue;
        const int64_t b = off[u], e = off[u + 1];
        const int64_t inside = pin[e] - pin[b];
        const int64_t as = kt[u];
        if (as) wself[u] += as;
        const int64_t self = wself[u] + 2 * inside;
        cnt_out[cmap[u]] = run[e] - run[b] + (self > 0 ? 1 : 0);
        kt[u] = k_in[u] + inside + as;
    }
}

// the kept entries into the coarse rows (after the self-loop's slot where the
// row passes its own vertex)
template <int WK>
__global__ __launch_bounds__(BLOCK) void k_vf_write(Csr g, const int32_t *cmap, const int32_t *A, const int64_t *run,
                                                    const int64_t *pin, const int64_t *wself, const int64_t *off_out,
                                                    int32_t *col_out, int64_t *w_out)
{
    __shared__ int64_t s_off[ROWCAP + 1];
    __shared__ int64_t s_meta[2];
    const int64_t e0 = (int64_t)blockIdx.x * ETILE;
    const int64_t e1 = min(e0 + ETILE, g.nnz) - 1;
    TileRows t = tile_rows(g.off, g.n, e0, e1, s_off, s_meta);
    for (int r = 0; r < EITEMS; ++r) {
        const int64_t e = e0 + r * BLOCK + threadIdx.x;
        if (e > e1) break;
        const int32_t a = A[e];
        if (a < 0) continue;
        const int64_t u = tile_row(t, g.off, s_off, e);
        const int64_t b = tile_off(t, g.off, s_off, u), en = tile_off(t, g.off, s_off, u + 1);
        const int64_t self = wself[u] + 2 * (pin[en] - pin[b]);
        const int64_t pos = off_out[cmap[u]] + (run[e] - run[b]) + ((self > 0 && g.col[e] > u) ? 1 : 0);
        col_out[pos] = a;
        w_out[pos] = WLoad<WK>::at(g.w, e);
    }
}

// coarse degrees, and each community's self-loop at its sorted place; 2m and
// the self-loop total into the replicated counters 0 and 2
__global__ __launch_bounds__(BLOCK) void k_vf_self(const int64_t *off, const int32_t *col, int64_t n,
                                                   const int32_t *map, const int32_t *cmap, const int64_t *run,
                                                   const int64_t *pin, const int64_t *wself, const int64_t *kt,
                                                   const int64_t *off_out, int32_t *col_out, int64_t *w_out,
                                                   int64_t *k_out, int64_t *rep)
{
    __shared__ int64_t s_red[BLOCK / 64];
    int64_t two = 0, selft = 0;
    for (int64_t u = (int64_t)blockIdx.x * BLOCK + threadIdx.x; u < n; u += (int64_t)gridDim.x * BLOCK) {
        if (map[u] != u) continue;
        const int32_t cu = cmap[u];
        const int64_t b = off[u], e = off[u + 1];
        const int64_t self = wself[u] + 2 * (pin[e] - pin[b]);
        k_out[cu] = kt[u];
        two += kt[u];
        if (self > 0) {
            int64_t lo = b, hi = e; // first entry of the row with a column above u
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (col[mid] <= u) lo = mid + 1;
                else hi = mid;
            }
            const int64_t pos = off_out[cu] + run[lo] - run[b];
            col_out[pos] = cu;
            w_out[pos] = self;
            selft += self;
        }
    }
    two = block_total(two, s_red);
    selft = block_total(selft, s_red);
    if (threadIdx.x == 0) {
        rep_add(rep, 0, two);
        rep_add(rep, 2, selft);
    }
}

hipError_t coarsen_vf(const Csr &g, const int32_t *map, const int64_t *k_in, int32_t *orig_map, int64_t n_orig,
                      CoarsenBufs &b, int64_t *off_out, int32_t *col_out, int64_t *w_out, int64_t *k_out,
                      int64_t *stats, int64_t *n_new, int64_t *nnz_new, Scratch &s, hipStream_t st)
{
    fill<int64_t>(stats, 0, 3, st);
    const int64_t n = g.n, nnz = g.nnz;
    // renumber the kept vertices (every community's label) in ascending id
    fill<int32_t>(b.flag, 0, n + 1, st);
    unsigned gv = grid_for(n, BLOCK * 4);
    if (gv > 65536) gv = 65536;
    if (n > 0) k_mark<<<gv, BLOCK, 0, st>>>(map, n, b.flag);
    scan_i32_to_i32(b.flag, b.new_id, n, s.scalar, s, st);
    int64_t nn = 0;
    if (const hipError_t e = read_back(&nn, s.scalar, st)) return e;
    unsigned gx = grid_for(n_orig, BLOCK * 4);
    if (gx > 65536) gx = 65536;
    if (n_orig > 0) k_compose<<<gx, BLOCK, 0, st>>>(orig_map, n_orig, map, b.new_id);
    *n_new = nn;
    if (nnz == 0) {
        fill<int64_t>(off_out, 0, nn + 1, st);
        fill<int64_t>(k_out, 0, nn, st);
        *nnz_new = 0;
        return hipGetLastError();
    }
    // the kept-vertex bitmap and word prefixes behind A in the keys buffer
    // when they fit there (A takes half a word per entry); else every
    // neighbour's id comes from cmap
    int32_t *A = (int32_t *)b.keys;
    const int64_t nw = (n + 63) / 64, a_words = (nnz + 1) / 2 + 1;
    uint64_t *kbits = nullptr;
    int32_t *kpre = nullptr;
    if (a_words + nw + (nw + 1) / 2 <= b.keys_words) {
        kbits = b.keys + a_words;
        kpre = (int32_t *)(kbits + nw);
        const int64_t gbw = (nw * 64 + BLOCK - 1) / BLOCK;
        k_keep_bits<<<(unsigned)(gbw < 65536 ? gbw : 65536), BLOCK, 0, st>>>(b.flag, b.new_id, n, kbits, kpre);
    }
    int32_t *cmap = b.flag; // free after the renumbering scan and the bitmap
    k_cmap<<<gv, BLOCK, 0, st>>>(map, b.new_id, n, cmap);
    int64_t *run = b.vals_alt, *pin = b.vals, *wself = b.run, *kt = (int64_t *)b.keys_alt;
    fill<int64_t>(wself, 0, n, st);
    fill<int64_t>(kt, 0, n, st); // absorbed self-loops first, then the community degrees
    const unsigned ge = grid_for(nnz, ETILE);
    switch (g.wk) {
    case W_UNIT: k_vf_entries<W_UNIT><<<ge, BLOCK, 0, st>>>(g, map, cmap, kbits, kpre, A, wself, kt); break;
    case W_I32: k_vf_entries<W_I32><<<ge, BLOCK, 0, st>>>(g, map, cmap, kbits, kpre, A, wself, kt); break;
    default: k_vf_entries<W_I64><<<ge, BLOCK, 0, st>>>(g, map, cmap, kbits, kpre, A, wself, kt); break;
    }
    scan_nonneg(A, run, nnz, run + nnz, s, st);
    scan_tagged_weights(A, VF_INSIDE, g.w, g.wk, pin, nnz, pin + nnz, s, st);
    k_vf_rows<<<gv, BLOCK, 0, st>>>(g.off, n, map, cmap, run, pin, wself, k_in, off_out, kt);
    scan_i64(off_out, off_out, nn, off_out + nn, s, st); // in place; the total is nnz'
    int64_t tot = 0;
    if (const hipError_t e = hipMemcpyAsync(&tot, off_out + nn, sizeof(int64_t), hipMemcpyDeviceToHost, st)) return e;
    switch (g.wk) {
    case W_UNIT: k_vf_write<W_UNIT><<<ge, BLOCK, 0, st>>>(g, cmap, A, run, pin, wself, off_out, col_out, w_out); break;
    case W_I32: k_vf_write<W_I32><<<ge, BLOCK, 0, st>>>(g, cmap, A, run, pin, wself, off_out, col_out, w_out); break;
    default: k_vf_write<W_I64><<<ge, BLOCK, 0, st>>>(g, cmap, A, run, pin, wself, off_out, col_out, w_out); break;
    }
    rep_clear(s.rep, st);
    k_vf_self<<<gv, BLOCK, 0, st>>>(g.off, g.col, n, map, cmap, run, pin, wself, kt, off_out, col_out, w_out, k_out,
                                    s.rep);
    rep_fold(s.rep, 3, stats, st); // 2m, 0 (the maximum below), self-loop total
    if (nn > 0) {
        unsigned gm = grid_for(nn, BLOCK * 16);
        if (gm > 4096) gm = 4096;
        k_max<<<gm, BLOCK, 0, st>>>(k_out, nn, stats + 1);
    }
    if (const hipError_t e = hipStreamSynchronize(st)) return e;
    *nnz_new = tot;
    return hipGetLastError();
}

template <int WK>
__global__ __launch_bounds__(BLOCK) void k_w64(const void *w, int64_t nnz, int64_t *out)
{
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * BLOCK)
        out[e] = WLoad<WK>::at(w, e);
}

void weights_i64(const Csr &g, int64_t *w_out, hipStream_t st)
{
    if (g.nnz == 0) return;
    unsigned gw = grid_for(g.nnz, BLOCK * 4);
    if (gw > 65536) gw = 65536;
    switch (g.wk) {
    case W_UNIT: k_w64<W_UNIT><<<gw, BLOCK, 0, st>>>(g.w, g.nnz, w_out); break;
    case W_I32: k_w64<W_I32><<<gw, BLOCK, 0, st>>>(g.w, g.nnz, w_out); break;
    default: k_w64<W_I64><<<gw, BLOCK, 0, st>>>(g.w, g.nnz, w_out); break;
    }
}

} // namespace lv
