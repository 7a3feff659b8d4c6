// Kernels of the batched form: many independent graphs packed as one
// disjoint-union CSR (graph g owns the contiguous vertex range
// [goff[g], goff[g+1]) and only edges inside it).  Sweeps, community updates
// and rebuilds run once over the union; the kernels here provide the
// per-graph pieces: graph ids, per-graph sums (2m, sum k^2, self-loops,
// sum a^2), commits restricted to the graphs that keep their iteration, and
// graph boundaries after a rebuild.
#include "lv.h"

namespace lv {

// graph id of every vertex (binary search over the graph offsets)
__global__ __launch_bounds__(BLOCK) void k_graph_ids(const int64_t *goff, int32_t ng, int64_t n, int32_t *gid)
{
    for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * BLOCK) {
        int32_t lo = 0, hi = ng;
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (goff[mid] <= v) lo = mid; else hi = mid;
        }
        gid[v] = lo;
    }
}

void graph_ids(const int64_t *goff, int32_t ng, int64_t n, int32_t *gid, hipStream_t st)
{
    if (n == 0) return;
    unsigned g = grid_for(n, BLOCK * 4);
    if (g > 65536) g = 65536;
    k_graph_ids<<<g, BLOCK, 0, st>>>(goff, ng, n, gid);
}

// entries whose endpoints lie in different graphs (any count > 0 is an error)
__global__ __launch_bounds__(BLOCK) void k_cross_edges(Csr g, const int32_t *gid, int32_t *flag)
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
        if (gid[u] != gid[g.col[e]]) atomicCAS(flag, 0, 6);
    }
}

void cross_edges(const Csr &g, const int32_t *gid, int32_t *flag, hipStream_t st)
{
    if (g.nnz == 0) return;
    k_cross_edges<<<grid_for(g.nnz, ETILE), BLOCK, 0, st>>>(g, gid, flag);
}

// 128-bit unsigned add into (lo, hi) words with 64-bit atomics: the carry of
// every low-word addition is added to the high word, so concurrent adds sum
// exactly
__device__ __forceinline__ void atomic_add_u128(unsigned long long *w, u128 v)
{
    const unsigned long long lo = (unsigned long long)v, hi = (unsigned long long)(v >> 64);
    const unsigned long long old = atomicAdd(&w[0], lo);
    const unsigned long long add_hi = hi + (old + lo < old ? 1ull : 0ull);
    if (add_hi) atomicAdd(&w[1], add_hi);
}

// per graph: out[4g..4g+3] = sum x, sum x^2 (lo, hi), sum of self-loop
// weights (if g.off) over the graph's vertices.  One block per tile of
// GS_TILE vertices (graphs are contiguous vertex ranges, so a tile meets
// consecutive graphs): a tile inside one graph is reduced in registers, a
// tile meeting up to GS_RUNS graphs in LDS, otherwise per vertex; every
// block then adds its partial sums to the graphs' totals.
constexpr int GS_TILE = 1024;
constexpr int GS_RUNS = 64;

template <int WK>
__global__ __launch_bounds__(BLOCK) void k_graph_sums(Csr g, const int64_t *x, const int32_t *gid, int64_t n,
                                                      unsigned long long *out)
{
    __shared__ unsigned long long acc[GS_RUNS][4];
    __shared__ u128 red[BLOCK];
    const int64_t v0 = (int64_t)blockIdx.x * GS_TILE;
    const int64_t v1 = min(v0 + (int64_t)GS_TILE, n);
    const int32_t g0 = gid[v0], g1 = gid[v1 - 1];
    const int mode = g0 == g1 ? 0 : (g1 - g0 < GS_RUNS ? 1 : 2);
    for (int i = threadIdx.x; i < GS_RUNS * 4; i += BLOCK) (&acc[0][0])[i] = 0;
    __syncthreads();
    u128 sum = 0, sq = 0, self = 0;
    for (int64_t v = v0 + threadIdx.x; v < v1; v += BLOCK) {
        const int64_t xv = x[v];
        const u128 q = (u128)((i128)xv * xv);
        int64_t sv = 0;
        if (g.off) {
            int64_t lo = g.off[v], hi = g.off[v + 1];
            while (lo < hi) { // self-loop entry of row v, if any (columns ascending)
                const int64_t mid = (lo + hi) >> 1;
                const int32_t c = g.col[mid];
                if (c == v) {
                    sv = WLoad<WK>::at(g.w, mid);
                    break;
                }
                if (c < v) lo = mid + 1; else hi = mid;
            }
        }
        if (mode == 0) {
            sum += (u128)xv;
            sq += q;
            self += (u128)sv;
        } else {
            unsigned long long *d = mode == 1 ? acc[gid[v] - g0] : out + 4 * (int64_t)gid[v];
            atomicAdd(&d[0], (unsigned long long)xv);
            atomic_add_u128(&d[1], q);
            if (sv) atomicAdd(&d[3], (unsigned long long)sv);
        }
    }
    if (mode == 0) {
        // block totals, one add per word
        u128 t[3] = {sum, sq, self};
        for (int k = 0; k < 3; ++k) {
            red[threadIdx.x] = t[k];
            __syncthreads();
            for (int h = BLOCK / 2; h > 0; h >>= 1) {
                if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
                __syncthreads();
            }
            t[k] = red[0];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            unsigned long long *d = out + 4 * (int64_t)g0;
            if ((uint64_t)t[0]) atomicAdd(&d[0], (unsigned long long)t[0]);
            atomic_add_u128(&d[1], t[1]);
            if ((uint64_t)t[2]) atomicAdd(&d[3], (unsigned long long)t[2]);
        }
        return;
    }
    __syncthreads();
    if (mode == 1)
        for (int r = threadIdx.x; r <= g1 - g0; r += BLOCK) {
            unsigned long long *d = out + 4 * (int64_t)(g0 + r);
            if (acc[r][0]) atomicAdd(&d[0], acc[r][0]);
            atomic_add_u128(&d[1], ((u128)acc[r][2] << 64) | (u128)acc[r][1]);
            if (acc[r][3]) atomicAdd(&d[3], acc[r][3]);
        }
}

void graph_sums(const Csr &g, bool with_self, const int64_t *x, const int32_t *gid, int32_t ng, int64_t *out,
                hipStream_t st)
{
    if (ng <= 0) return;
    fill<int64_t>(out, 0, 4 * (int64_t)ng, st);
    if (g.n <= 0) return;
    Csr c = g;
    if (!with_self) c.off = nullptr;
    const unsigned blocks = grid_for(g.n, GS_TILE);
    unsigned long long *o = (unsigned long long *)out;
    switch (g.wk) {
    case W_UNIT: k_graph_sums<W_UNIT><<<blocks, BLOCK, 0, st>>>(c, x, gid, g.n, o); break;
    case W_I32: k_graph_sums<W_I32><<<blocks, BLOCK, 0, st>>>(c, x, gid, g.n, o); break;
    default: k_graph_sums<W_I64><<<blocks, BLOCK, 0, st>>>(c, x, gid, g.n, o); break;
    }
}

// per graph g, by mode[g]: 1 commits the sweep's moves and keeps the
// partition they replace in comm_save; 2 undoes the last committed iteration
// (every vertex back to comm_save, Sec. 5.1: a loss ends the phase and is not
// kept); 0 drops the sweep's proposals (comm_next reset to comm_prev)
__global__ __launch_bounds__(BLOCK) void k_commit_graphs(int64_t n, int32_t *comm_prev, int32_t *comm_next,
                                                         int32_t *comm_save, const int64_t *k, int64_t *a,
                                                         int32_t *size, const int32_t *gid, const int32_t *mode)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        const int32_t m = mode[gid[i]];
        const int32_t A = comm_prev[i];
        int32_t B;
        if (m == 1) {
            B = comm_next[i];
            comm_save[i] = A;
        } else if (m == 2) {
            B = comm_save[i];
            if (comm_next[i] != B) comm_next[i] = B;
        } else {
            if (comm_next[i] != A) comm_next[i] = A;
            continue;
        }
        if (A == B) continue;
        const int64_t ki = k[i];
        atomicAdd((unsigned long long *)&a[A], (unsigned long long)(-ki));
        atomicAdd((unsigned long long *)&a[B], (unsigned long long)ki);
        atomicSub(&size[A], 1);
        atomicAdd(&size[B], 1);
        comm_prev[i] = B;
    }
}

void commit_graphs(int64_t n, int32_t *comm_prev, int32_t *comm_next, int32_t *comm_save, const int64_t *k,
                   int64_t *a, int32_t *size, const int32_t *gid, const int32_t *mode, hipStream_t st)
{
    if (n <= 0) return;
    unsigned gc = grid_for(n, BLOCK * 4);
    if (gc > 65536) gc = 65536;
    k_commit_graphs<<<gc, BLOCK, 0, st>>>(n, comm_prev, comm_next, comm_save, k, a, size, gid, mode);
}

// graph boundaries after a rebuild: new_goff[g] = new id of the first vertex
// of graph g (new_id is the exclusive prefix of non-empty communities, whose
// order follows the graphs), new_goff[ng] = total
__global__ __launch_bounds__(BLOCK) void k_new_goff(const int64_t *goff, int32_t ng, int64_t n, const int32_t *new_id,
                                                    int64_t total, int64_t *new_goff)
{
    for (int64_t g = (int64_t)blockIdx.x * BLOCK + threadIdx.x; g <= ng; g += (int64_t)gridDim.x * BLOCK)
        new_goff[g] = goff[g] < n ? (int64_t)new_id[goff[g]] : total;
}

void new_graph_offsets(const int64_t *goff, int32_t ng, int64_t n, const int32_t *new_id, int64_t total,
                       int64_t *new_goff, hipStream_t st)
{
    k_new_goff<<<grid_for(ng + 1, BLOCK), BLOCK, 0, st>>>(goff, ng, n, new_id, total, new_goff);
}

// union CSR assembled from per-graph arrays copied side by side: every
// offset gets its graph's first entry index, every column its graph's first
// vertex id (eoff: graphs' first entries; graph of an entry = the last graph
// whose first entry is at or before it, so empty graphs are skipped)
__global__ __launch_bounds__(BLOCK) void k_batch_fixup(int64_t *off, int64_t n, int32_t *col, int64_t nnz,
                                                       const int64_t *goff, const int64_t *eoff, int32_t ng)
{
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += stride) {
        int32_t lo = 0, hi = ng;
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (goff[mid] <= v) lo = mid; else hi = mid;
        }
        off[v] += eoff[lo];
    }
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < nnz; e += stride) {
        int32_t lo = 0, hi = ng;
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (eoff[mid] <= e) lo = mid; else hi = mid;
        }
        col[e] += (int32_t)goff[lo];
    }
}

void batch_fixup(int64_t *off, int64_t n, int32_t *col, int64_t nnz, const int64_t *goff, const int64_t *eoff,
                 int32_t ng, hipStream_t st)
{
    if (ng <= 0 || (n <= 0 && nnz <= 0)) return;
    unsigned g = grid_for(n > nnz ? n : nnz, BLOCK * 4);
    if (g > 65536) g = 65536;
    k_batch_fixup<<<g, BLOCK, 0, st>>>(off, n, col, nnz, goff, eoff, ng);
}

// local labels: label[x] = orig_map[x] - goff[graph of x]
__global__ __launch_bounds__(BLOCK) void k_local_labels(const int32_t *orig_map, const int32_t *gid0, int64_t n0,
                                                        const int64_t *goff, int32_t *labels)
{
    for (int64_t x = (int64_t)blockIdx.x * BLOCK + threadIdx.x; x < n0; x += (int64_t)gridDim.x * BLOCK)
        labels[x] = (int32_t)(orig_map[x] - goff[gid0[x]]);
}

void local_labels(const int32_t *orig_map, const int32_t *gid0, int64_t n0, const int64_t *goff, int32_t *labels,
                  hipStream_t st)
{
    if (n0 == 0) return;
    unsigned g = grid_for(n0, BLOCK * 4);
    if (g > 65536) g = 65536;
    k_local_labels<<<g, BLOCK, 0, st>>>(orig_map, gid0, n0, goff, labels);
}

} // namespace lv
