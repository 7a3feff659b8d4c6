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

__device__ __forceinline__ u128 block_sum_u128(u128 v, u128 *s)
{
    s[threadIdx.x] = v;
    __syncthreads();
    for (int h = BLOCK / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    const u128 r = s[0];
    __syncthreads();
    return r;
}

// per graph (one block each): out[4g..4g+3] = sum x (int64), sum x^2 (lo, hi),
// sum of self-loop weights (int64), over the graph's vertices
template <int WK>
__global__ __launch_bounds__(BLOCK) void k_graph_sums(Csr g, const int64_t *x, const int64_t *goff, int64_t *out)
{
    __shared__ u128 s[BLOCK];
    const int64_t gi = blockIdx.x;
    const int64_t b = goff[gi], e = goff[gi + 1];
    u128 sum = 0, sq = 0, self = 0;
    for (int64_t v = b + threadIdx.x; v < e; v += BLOCK) {
        const int64_t xv = x[v];
        sum += (u128)xv;
        sq += (u128)((i128)xv * xv);
        if (g.off) {
            int64_t lo = g.off[v], hi = g.off[v + 1];
            while (lo < hi) { // self-loop entry of row v, if any
                const int64_t mid = (lo + hi) >> 1;
                const int32_t c = g.col[mid];
                if (c == v) {
                    self += (u128)WLoad<WK>::at(g.w, mid);
                    break;
                }
                if (c < v) lo = mid + 1; else hi = mid;
            }
        }
    }
    sum = block_sum_u128(sum, s);
    sq = block_sum_u128(sq, s);
    self = block_sum_u128(self, s);
    if (threadIdx.x == 0) {
        out[4 * gi + 0] = (int64_t)(uint64_t)sum;
        out[4 * gi + 1] = (int64_t)(uint64_t)sq;
        out[4 * gi + 2] = (int64_t)(uint64_t)(sq >> 64);
        out[4 * gi + 3] = (int64_t)(uint64_t)self;
    }
}

void graph_sums(const Csr &g, bool with_self, const int64_t *x, const int64_t *goff, int32_t ng, int64_t *out,
                hipStream_t st)
{
    if (ng <= 0) return;
    Csr c = g;
    if (!with_self) c.off = nullptr;
    switch (g.wk) {
    case W_UNIT: k_graph_sums<W_UNIT><<<(unsigned)ng, BLOCK, 0, st>>>(c, x, goff, out); break;
    case W_I32: k_graph_sums<W_I32><<<(unsigned)ng, BLOCK, 0, st>>>(c, x, goff, out); break;
    default: k_graph_sums<W_I64><<<(unsigned)ng, BLOCK, 0, st>>>(c, x, goff, out); break;
    }
}

// commits the moves of graphs with keep[g] != 0; other graphs drop the
// sweep's proposals (comm_next reset to comm_prev)
__global__ __launch_bounds__(BLOCK) void k_commit_graphs(int64_t n, int32_t *comm_prev, int32_t *comm_next,
                                                         const int64_t *k, int64_t *a, int32_t *size,
                                                         const int32_t *gid, const int32_t *keep)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        const int32_t A = comm_prev[i], B = comm_next[i];
        if (A == B) continue;
        if (!keep[gid[i]]) {
            comm_next[i] = A;
            continue;
        }
        const int64_t ki = k[i];
        atomicAdd((unsigned long long *)&a[A], (unsigned long long)(-ki));
        atomicAdd((unsigned long long *)&a[B], (unsigned long long)ki);
        atomicSub(&size[A], 1);
        atomicAdd(&size[B], 1);
        comm_prev[i] = B;
    }
}

void commit_graphs(int64_t n, int32_t *comm_prev, int32_t *comm_next, const int64_t *k, int64_t *a, int32_t *size,
                   const int32_t *gid, const int32_t *keep, hipStream_t st)
{
    if (n <= 0) return;
    unsigned gc = grid_for(n, BLOCK * 4);
    if (gc > 65536) gc = 65536;
    k_commit_graphs<<<gc, BLOCK, 0, st>>>(n, comm_prev, comm_next, k, a, size, gid, keep);
}

// per graph (one block each): internal weight of its current partition
template <int WK>
__global__ __launch_bounds__(BLOCK) void k_graph_internal(Csr g, const int32_t *comm, const int64_t *goff, int64_t *out)
{
    __shared__ u128 s[BLOCK];
    const int64_t gi = blockIdx.x;
    u128 acc = 0;
    for (int64_t v = goff[gi] + threadIdx.x; v < goff[gi + 1]; v += BLOCK)
        for (int64_t e = g.off[v]; e < g.off[v + 1]; ++e)
            if (comm[g.col[e]] == comm[v]) acc += (u128)WLoad<WK>::at(g.w, e);
    acc = block_sum_u128(acc, s);
    if (threadIdx.x == 0) out[gi] = (int64_t)(uint64_t)acc;
}

void graph_internal(const Csr &g, const int32_t *comm, const int64_t *goff, int32_t ng, int64_t *out, hipStream_t st)
{
    if (ng <= 0) return;
    switch (g.wk) {
    case W_UNIT: k_graph_internal<W_UNIT><<<(unsigned)ng, BLOCK, 0, st>>>(g, comm, goff, out); break;
    case W_I32: k_graph_internal<W_I32><<<(unsigned)ng, BLOCK, 0, st>>>(g, comm, goff, out); break;
    default: k_graph_internal<W_I64><<<(unsigned)ng, BLOCK, 0, st>>>(g, comm, goff, out); break;
    }
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
