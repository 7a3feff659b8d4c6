/*
 * Seeded synthetic graph generators: planted-partition SBM, R-MAT and
 * weighted Chung-Lu.  These stand in for the paper's input families
 * (citation/collaboration graphs, internet/social graphs and the weighted
 * metagenomic similarity graphs of Table 1).
 *
 * This module holds no arithmetic of the community-detection method; it only
 * produces inputs.  Every random number comes from the counter-based
 * Philox4x32-10 generator (Salmon, Moraes, Dror, Shaw, SC'11) keyed by
 * (seed, stream) and indexed by the position of the draw, so the output is a
 * pure function of the arguments and never depends on the thread count.
 *
 * Output: an undirected graph as a symmetric CSR (int64 offsets, int32
 * columns sorted ascending and unique per row, int32 weights >= 1 or no weight
 * array for unit weights).  No self-loops are generated.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct {
    int64_t n, nnz;
    int64_t *off;   /* n+1 */
    int32_t *col;   /* nnz */
    int32_t *w;     /* nnz, NULL = unit weights */
} gg_csr;

/* ------------------------------------------------------------------ */
/* Philox4x32-10                                                        */
/* ------------------------------------------------------------------ */
static inline void philox4x32_10(const uint32_t in[4], uint32_t k0, uint32_t k1, uint32_t out[4])
{
    uint32_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* exported for a known-answer test of the generator's PRNG */
void gg_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    philox4x32_10(ctr, key[0], key[1], out);
}

/* four 32-bit words for draw (i, j) of stream `stream` */
static inline void draw4(uint64_t seed, uint32_t stream, uint64_t i, uint32_t j, uint32_t out[4])
{
    uint32_t c[4] = { (uint32_t)i, (uint32_t)(i >> 32), j, stream };
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32), out);
}

/* uniform double in (0, 1] from two words (53 bits) */
static inline double u01_open0(uint32_t a, uint32_t b)
{
    uint64_t x = ((uint64_t)a << 32) | b;
    return ((double)(x >> 11) + 1.0) * (1.0 / 9007199254740992.0);
}

/* uniform integer in [lo, hi] from one word (multiply-shift) */
static inline int64_t uint_range(uint32_t r, int64_t lo, int64_t hi)
{
    uint64_t span = (uint64_t)(hi - lo + 1);
    return lo + (int64_t)(((uint64_t)r * span) >> 32);
}

/* ------------------------------------------------------------------ */
/* undirected edge list -> symmetric CSR                               */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t cnt, cap;
    uint32_t *u, *v, *w;
} edge_buf;

static void eb_push(edge_buf *b, uint32_t u, uint32_t v, uint32_t w)
{
    if (b->cnt == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 1024;
        b->u = (uint32_t *)realloc(b->u, b->cap * sizeof(uint32_t));
        b->v = (uint32_t *)realloc(b->v, b->cap * sizeof(uint32_t));
        b->w = (uint32_t *)realloc(b->w, b->cap * sizeof(uint32_t));
    }
    b->u[b->cnt] = u; b->v[b->cnt] = v; b->w[b->cnt] = w; b->cnt++;
}

static void eb_free(edge_buf *b) { free(b->u); free(b->v); free(b->w); memset(b, 0, sizeof(*b)); }

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/*
 * Builds the symmetric CSR of E undirected edges (eu[e], ev[e], ew[e]),
 * eu != ev.  Duplicate pairs are merged keeping the smallest weight, so the
 * result does not depend on the order of the list.  ew == NULL => unit weights.
 */
static gg_csr *build_csr(int64_t n, int64_t E, const uint32_t *eu, const uint32_t *ev,
                         const uint32_t *ew)
{
    int64_t *deg = (int64_t *)calloc(n + 1, sizeof(int64_t));
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
#pragma omp atomic
        deg[eu[e]]++;
#pragma omp atomic
        deg[ev[e]]++;
    }
    int64_t *off = (int64_t *)malloc((n + 1) * sizeof(int64_t));
    off[0] = 0;
    for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + deg[i];
    int64_t tot = off[n];
    uint64_t *ent = (uint64_t *)malloc((tot ? tot : 1) * sizeof(uint64_t));
    int64_t *cur = deg; /* reuse as cursor */
    memcpy(cur, off, n * sizeof(int64_t));
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        uint64_t w = ew ? ew[e] : 1u;
        int64_t p, q;
#pragma omp atomic capture
        p = cur[eu[e]]++;
#pragma omp atomic capture
        q = cur[ev[e]]++;
        ent[p] = ((uint64_t)ev[e] << 32) | w;
        ent[q] = ((uint64_t)eu[e] << 32) | w;
    }
    /* sort each row by (column, weight), then drop repeated columns */
    int64_t *keep = (int64_t *)malloc((n + 1) * sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
        uint64_t *r = ent + off[i];
        int64_t d = off[i + 1] - off[i];
        if (d > 1) qsort(r, d, sizeof(uint64_t), cmp_u64);
        int64_t k = 0;
        for (int64_t t = 0; t < d; ++t)
            if (k == 0 || (r[t] >> 32) != (r[k - 1] >> 32)) r[k++] = r[t];
        keep[i] = k;
    }
    gg_csr *g = (gg_csr *)calloc(1, sizeof(gg_csr));
    g->n = n;
    g->off = (int64_t *)malloc((n + 1) * sizeof(int64_t));
    g->off[0] = 0;
    for (int64_t i = 0; i < n; ++i) g->off[i + 1] = g->off[i] + keep[i];
    g->nnz = g->off[n];
    g->col = (int32_t *)malloc((g->nnz ? g->nnz : 1) * sizeof(int32_t));
    g->w = ew ? (int32_t *)malloc((g->nnz ? g->nnz : 1) * sizeof(int32_t)) : NULL;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
        const uint64_t *r = ent + off[i];
        int64_t o = g->off[i];
        for (int64_t t = 0; t < keep[i]; ++t) {
            g->col[o + t] = (int32_t)(r[t] >> 32);
            if (g->w) g->w[o + t] = (int32_t)(uint32_t)r[t];
        }
    }
    free(keep); free(ent); free(off); free(deg);
    return g;
}

/* ------------------------------------------------------------------ */
/* planted-partition SBM (geometric skip sampling per block pair)      */
/* ------------------------------------------------------------------ */
/*
 * n vertices in B blocks of near-equal size (the first n % B blocks get one
 * extra vertex; block b holds a contiguous id range).  Each unordered pair in
 * the same block is an edge with probability p_in, across blocks with p_out.
 * Weights are uniform in [1, wmax] (wmax <= 1 => unit, no weight array).
 */
gg_csr *gg_sbm(int64_t n, int32_t B, double p_in, double p_out, int32_t wmax,
               uint64_t seed, uint32_t stream)
{
    if (B < 1) B = 1;
    if (B > n) B = (int32_t)(n > 0 ? n : 1);
    int64_t *start = (int64_t *)malloc((B + 1) * sizeof(int64_t));
    start[0] = 0;
    for (int32_t b = 0; b < B; ++b) start[b + 1] = start[b] + n / B + (b < n % B ? 1 : 0);
    int64_t npairs = (int64_t)B * (B + 1) / 2;
    edge_buf *bufs = (edge_buf *)calloc(npairs, sizeof(edge_buf));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < npairs; ++q) {
        /* q -> (b1 <= b2), row-major over the upper triangle */
        int32_t b1 = 0;
        int64_t rem = q;
        while (rem >= B - b1) { rem -= B - b1; ++b1; }
        int32_t b2 = b1 + (int32_t)rem;
        double p = (b1 == b2) ? p_in : p_out;
        if (p <= 0.0) continue;
        int64_t s1 = start[b1 + 1] - start[b1], s2 = start[b2 + 1] - start[b2];
        int64_t total = s1 * s2; /* full rectangle; within a block keep only i < j */
        double lq = (p < 1.0) ? log1p(-p) : 0.0;
        int64_t idx = -1;
        for (uint32_t j = 0;; ++j) {
            uint32_t r[4];
            draw4(seed, stream, (uint64_t)q, j, r);
            if (p >= 1.0) idx += 1;
            else {
                double u = u01_open0(r[0], r[1]);
                double skip = floor(log(u) / lq);
                if (skip > (double)total) break;
                idx += 1 + (int64_t)skip;
            }
            if (idx >= total) break;
            int64_t a = start[b1] + idx / s2, c = start[b2] + idx % s2;
            if (b1 == b2 && a >= c) continue;
            uint32_t w = (wmax > 1) ? (uint32_t)uint_range(r[2], 1, wmax) : 1u;
            eb_push(&bufs[q], (uint32_t)a, (uint32_t)c, w);
        }
    }
    int64_t E = 0;
    for (int64_t q = 0; q < npairs; ++q) E += bufs[q].cnt;
    uint32_t *eu = (uint32_t *)malloc((E ? E : 1) * 4), *ev = (uint32_t *)malloc((E ? E : 1) * 4),
             *ew = (uint32_t *)malloc((E ? E : 1) * 4);
    int64_t o = 0;
    for (int64_t q = 0; q < npairs; ++q) {
        memcpy(eu + o, bufs[q].u, bufs[q].cnt * 4);
        memcpy(ev + o, bufs[q].v, bufs[q].cnt * 4);
        memcpy(ew + o, bufs[q].w, bufs[q].cnt * 4);
        o += bufs[q].cnt;
        eb_free(&bufs[q]);
    }
    free(bufs); free(start);
    gg_csr *g = build_csr(n, E, eu, ev, wmax > 1 ? ew : NULL);
    free(eu); free(ev); free(ew);
    return g;
}

/* ------------------------------------------------------------------ */
/* R-MAT                                                                */
/* ------------------------------------------------------------------ */
/* seeded Fisher-Yates permutation of [0, N) */
static void permutation(int64_t N, uint64_t seed, uint32_t stream, uint32_t *perm)
{
    for (int64_t i = 0; i < N; ++i) perm[i] = (uint32_t)i;
    for (int64_t i = N - 1; i > 0; --i) {
        uint32_t r[4];
        draw4(seed, stream, (uint64_t)i, 0, r);
        uint64_t x = ((uint64_t)r[0] << 32) | r[1];
        int64_t j = (int64_t)(((unsigned __int128)x * (uint64_t)(i + 1)) >> 64);
        uint32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
}

/*
 * R-MAT: edge_factor * 2^scale samples; each level picks a quadrant with
 * probabilities (a, b, c, 1-a-b-c).  Vertex ids are then relabelled by a
 * seeded random permutation; self-loops are dropped and duplicates merged.
 * n_keep > 0 keeps only edges whose relabelled endpoints are < n_keep (the
 * graph then has n_keep vertices).  Weights uniform in [1, wmax] per sample
 * (merged duplicates keep the smallest), wmax <= 1 => unit.
 */
gg_csr *gg_rmat(int32_t scale, int64_t edge_factor, double a, double b, double c,
                int32_t wmax, uint64_t seed, int64_t n_keep)
{
    int64_t N = (int64_t)1 << scale;
    int64_t S = edge_factor * N;
    int64_t n = (n_keep > 0 && n_keep < N) ? n_keep : N;
    uint32_t ta = (uint32_t)floor(a * 4294967296.0);
    uint32_t tb = (uint32_t)floor((a + b) * 4294967296.0);
    uint32_t tc = (uint32_t)floor((a + b + c) * 4294967296.0);
    uint32_t *perm = (uint32_t *)malloc(N * sizeof(uint32_t));
    permutation(N, seed, 1u, perm);
    uint32_t *eu = (uint32_t *)malloc(S * 4), *ev = (uint32_t *)malloc(S * 4);
    uint32_t *ew = (wmax > 1) ? (uint32_t *)malloc(S * 4) : NULL;
    uint8_t *ok = (uint8_t *)malloc(S);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < S; ++s) {
        uint32_t u = 0, v = 0, r[4];
        for (int32_t l = 0; l < scale; ++l) {
            if ((l & 3) == 0) draw4(seed, 2u, (uint64_t)s, (uint32_t)(l >> 2), r);
            uint32_t x = r[l & 3];
            uint32_t bu = (x >= tb), bv = (x >= ta && x < tb) || (x >= tc);
            u = (u << 1) | bu;
            v = (v << 1) | bv;
        }
        u = perm[u]; v = perm[v];
        eu[s] = u; ev[s] = v;
        ok[s] = (u != v) && (u < (uint64_t)n) && (v < (uint64_t)n);
        if (ew) {
            uint32_t q[4];
            draw4(seed, 3u, (uint64_t)s, 0, q);
            ew[s] = (uint32_t)uint_range(q[0], 1, wmax);
        }
    }
    /* compact kept samples (order-preserving, serial) */
    int64_t E = 0;
    for (int64_t s = 0; s < S; ++s)
        if (ok[s]) { eu[E] = eu[s]; ev[E] = ev[s]; if (ew) ew[E] = ew[s]; ++E; }
    free(ok); free(perm);
    gg_csr *g = build_csr(n, E, eu, ev, ew);
    free(eu); free(ev); free(ew);
    return g;
}

/* ------------------------------------------------------------------ */
/* weighted Chung-Lu                                                    */
/* ------------------------------------------------------------------ */
static double cl_mass(int64_t n, double beta, double i0)
{
    /* sum_{i<n} (i+i0)^-beta : first 4096 terms exactly, the rest by the midpoint rule */
    const int64_t K = n < 4096 ? n : 4096;
    double s = 0.0;
    for (int64_t i = 0; i < K; ++i) s += pow((double)i + i0, -beta);
    if (n > K) {
        double lo = (double)K - 0.5 + i0, hi = (double)n - 0.5 + i0;
        s += (pow(hi, 1.0 - beta) - pow(lo, 1.0 - beta)) / (1.0 - beta);
    }
    return s;
}

typedef struct { uint64_t key; int64_t idx; } kv_t;
static int cmp_kv(const void *a, const void *b)
{
    const kv_t *x = (const kv_t *)a, *y = (const kv_t *)b;
    if (x->key != y->key) return (x->key > y->key) - (x->key < y->key);
    return (x->idx > y->idx) - (x->idx < y->idx);
}
static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/*
 * Chung-Lu with expected-degree weights w_i = wtop * (i0 / (i + i0))^(1/(gamma-1)),
 * i0 chosen so that sum_i w_i = wsum.  Endpoint pairs are drawn independently
 * with probability proportional to w (inverse CDF); the first m_edges distinct
 * non-loop unordered pairs in draw order are kept.  Edge weights uniform in
 * [1, wmax] keyed by the pair's first draw index.
 */
gg_csr *gg_chung_lu(int64_t n, double gamma, double wtop, double wsum, int64_t m_edges,
                    int32_t wmax, uint64_t seed)
{
    double beta = 1.0 / (gamma - 1.0);
    /* bisection on log(i0): f(i0) = wtop * i0^beta * mass(i0) - wsum is increasing in i0 */
    double lo = -10.0, hi = 40.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi), i0 = exp(mid);
        double f = wtop * pow(i0, beta) * cl_mass(n, beta, i0) - wsum;
        if (f > 0) hi = mid; else lo = mid;
    }
    double i0 = exp(0.5 * (lo + hi));
    double *cdf = (double *)malloc((n + 1) * sizeof(double));
    cdf[0] = 0.0;
    for (int64_t i = 0; i < n; ++i) cdf[i + 1] = cdf[i] + pow(i0 / ((double)i + i0), beta);
    double total = cdf[n];

    int64_t S = m_edges + m_edges / 8 + 1024;
    for (;;) {
        kv_t *kv = (kv_t *)malloc(S * sizeof(kv_t));
#pragma omp parallel for schedule(static)
        for (int64_t s = 0; s < S; ++s) {
            uint32_t r[4];
            draw4(seed, 4u, (uint64_t)s, 0, r);
            double x1 = (u01_open0(r[0], r[1]) - 0x1p-53) * total;
            double x2 = (u01_open0(r[2], r[3]) - 0x1p-53) * total;
            int64_t e[2];
            double xs[2] = { x1, x2 };
            for (int t = 0; t < 2; ++t) { /* largest i with cdf[i] <= x */
                int64_t L = 0, H = n - 1;
                while (L < H) {
                    int64_t M = (L + H + 1) >> 1;
                    if (cdf[M] <= xs[t]) L = M; else H = M - 1;
                }
                e[t] = L;
            }
            int64_t u = e[0] < e[1] ? e[0] : e[1], v = e[0] < e[1] ? e[1] : e[0];
            kv[s].key = (u == v) ? UINT64_MAX : (((uint64_t)u << 32) | (uint64_t)v);
            kv[s].idx = s;
        }
        /* group by smaller endpoint (bucket), sort within bucket, keep first draw */
        int64_t *cnt = (int64_t *)calloc(n + 2, sizeof(int64_t));
        for (int64_t s = 0; s < S; ++s) {
            int64_t bkt = kv[s].key == UINT64_MAX ? n : (int64_t)(kv[s].key >> 32);
            cnt[bkt + 1]++;
        }
        for (int64_t i = 0; i < n + 1; ++i) cnt[i + 1] += cnt[i];
        kv_t *sorted = (kv_t *)malloc(S * sizeof(kv_t));
        int64_t *cur = (int64_t *)malloc((n + 1) * sizeof(int64_t));
        memcpy(cur, cnt, (n + 1) * sizeof(int64_t));
        for (int64_t s = 0; s < S; ++s) {
            int64_t bkt = kv[s].key == UINT64_MAX ? n : (int64_t)(kv[s].key >> 32);
            sorted[cur[bkt]++] = kv[s];
        }
        free(cur); free(kv);
        int64_t *firsts = (int64_t *)malloc(S * sizeof(int64_t));
        int64_t U = 0;
#pragma omp parallel for schedule(dynamic, 4096)
        for (int64_t i = 0; i < n; ++i) {
            kv_t *r = sorted + cnt[i];
            int64_t d = cnt[i + 1] - cnt[i];
            if (d > 1) qsort(r, d, sizeof(kv_t), cmp_kv);
        }
        /* sorted by (key, draw index): the first of each run of equal keys is its first draw */
        for (int64_t s = 0; s < cnt[n]; ++s)
            if (s == 0 || sorted[s - 1].key != sorted[s].key) firsts[U++] = sorted[s].idx;
        if (U < m_edges) {
            free(firsts); free(sorted); free(cnt);
            S = S + S / 4;
            continue;
        }
        int64_t *tmp = (int64_t *)malloc(U * sizeof(int64_t));
        memcpy(tmp, firsts, U * sizeof(int64_t));
        qsort(tmp, U, sizeof(int64_t), cmp_i64);
        int64_t cut = tmp[m_edges - 1];
        free(tmp);
        uint32_t *eu = (uint32_t *)malloc(m_edges * 4), *ev = (uint32_t *)malloc(m_edges * 4),
                 *ew = (uint32_t *)malloc(m_edges * 4);
        int64_t E = 0;
        for (int64_t s = 0; s < cnt[n]; ++s) {
            if (s > 0 && sorted[s - 1].key == sorted[s].key) continue;
            if (sorted[s].idx > cut) continue;
            uint32_t q[4];
            draw4(seed, 5u, (uint64_t)sorted[s].idx, 0, q);
            eu[E] = (uint32_t)(sorted[s].key >> 32);
            ev[E] = (uint32_t)sorted[s].key;
            ew[E] = (wmax > 1) ? (uint32_t)uint_range(q[0], 1, wmax) : 1u;
            ++E;
        }
        free(firsts); free(sorted); free(cnt); free(cdf);
        gg_csr *g = build_csr(n, E, eu, ev, wmax > 1 ? ew : NULL);
        free(eu); free(ev); free(ew);
        return g;
    }
}

/* ------------------------------------------------------------------ */
/* per-graph parameter draws for batched / served mixes                 */
/* ------------------------------------------------------------------ */
/* four uniform doubles in (0,1] for (seed, stream, index) */
void gg_uniform4(uint64_t seed, uint32_t stream, uint64_t index, double out[4])
{
    uint32_t r[4], q[4];
    draw4(seed, stream, index, 0, r);
    draw4(seed, stream, index, 1, q);
    out[0] = u01_open0(r[0], r[1]);
    out[1] = u01_open0(r[2], r[3]);
    out[2] = u01_open0(q[0], q[1]);
    out[3] = u01_open0(q[2], q[3]);
}

/* ------------------------------------------------------------------ */
/* accessors                                                            */
/* ------------------------------------------------------------------ */
void gg_info(const gg_csr *g, int64_t out[3])
{
    out[0] = g->n;
    out[1] = g->nnz;
    out[2] = g->w ? 1 : 0;
}

void gg_copy(const gg_csr *g, int64_t *off, int32_t *col, int32_t *w)
{
    memcpy(off, g->off, (g->n + 1) * sizeof(int64_t));
    if (g->nnz) memcpy(col, g->col, g->nnz * sizeof(int32_t));
    if (w && g->w && g->nnz) memcpy(w, g->w, g->nnz * sizeof(int32_t));
}

void gg_free(gg_csr *g)
{
    if (!g) return;
    free(g->off); free(g->col); free(g->w); free(g);
}
