/*
 * ORACLE -- test infrastructure only.
 *
 * A plain, slow, serial CPU implementation of the synchronous parallel
 * Louvain heuristic of Lu, Halappanavar and Kalyanaraman ("Parallel
 * heuristics for scalable community detection"), used to check the GPU
 * library bit for bit.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never does.  It shares
 * no code, header, table or helper with the GPU library.
 *
 * Arithmetic is exact: integer edge weights, int64 degrees, __int128 gains
 * and modularity numerators.  Every data structure is the simplest that is
 * obviously right (std::map per vertex for neighbouring communities,
 * std::map keyed by community pairs for coarsening, a sort by priority for
 * coloring).
 *
 * Readings of the paper fixed here (the GPU library follows the same ones):
 *  - degrees and modularity (Sec. 2, Eq. 2-3): a self-loop is stored once in
 *    the CSR and counts once in k_i, in e_{i->C(i)} and in the internal weight;
 *    with that convention Eq. 3 and Eq. 4 agree exactly.
 *  - gain (Sec. 3, Eq. 4): for vertex i in community A and candidate c != A,
 *    2m^2 * dQ = G(c) - G_stay with G(c) = 2m*e_{i->c} - k_i*a_c and
 *    G_stay = 2m*e_{i->A\{i}} - k_i*(a_A - k_i).  Staying has gain 0.
 *  - target (Eq. 5, Alg. 1 inner loop): lexicographic max of (G(c), -c) over
 *    the communities of i's non-self neighbours other than A (minimum-label
 *    tie-break, Sec. 5.1); move iff G(c*) > G_stay strictly.
 *  - singlet minimum-label heuristic (Sec. 5.1): a vertex alone in A does
 *    not move to a one-vertex community c* with a larger label; it then stays
 *    (no fallback to the second best).
 *  - synchronous sweep (Sec. 5.4 step 3): all decisions of an iteration read
 *    the state left by the previous iteration; with coloring, classes are
 *    processed in ascending color and each class reads the state left by the
 *    classes before it.
 *  - iteration stop (Alg. 1 threshold test, read with Sec. 5.1's remark that a
 *    minimum net gain is required to continue a phase): an iteration that
 *    loses modularity (Q_t < Q_{t-1}, where Q_0 is the phase's starting
 *    partition) is not a net gain: it is undone and ends the phase (Lemma 1
 *    of Sec. 4.1: simultaneous moves can lose).  Otherwise, from the second
 *    iteration on, stop when Q_t - Q_{t-1} < theta * |Q_{t-1}| (Alg. 1
 *    starts from Q_P = -infinity, so the first iteration never meets the
 *    test; the absolute value of Alg. 1 would never stop a two-state swap
 *    oscillation); also when an iteration moves nothing or the iteration
 *    cap is hit.  The moves of an iteration that gains are kept.  So no
 *    phase ends below the modularity it started from.
 *  - coarsening (Sec. 3, Sec. 5.5): non-empty communities renumbered in
 *    ascending id; coarse weight W'(C,D) = sum of all CSR entries from C to D,
 *    so an internal undirected edge contributes twice to the coarse self-loop.
 *  - vertex following (Sec. 5.3): a vertex whose row is exactly one entry
 *    (i,j), j != i, merges into j; an isolated pair merges into the smaller
 *    id; applied once, before the first phase.
 *  - chain-compressing vertex following (the extension closing Sec. 5.3):
 *    rounds of the same merge for single-neighbour vertices (one neighbour
 *    j != i, a self-loop allowed), each taken only while the bound in the
 *    proof of Lemma 3 stays positive, 2m * w_ij > k_i * k_j (the exact gain
 *    of moving i into j's one-vertex community, Eq. 4); every round rebuilds
 *    the graph, and the rounds repeat until no vertex qualifies.
 *  - coloring (Sec. 5.2): distance-1, greedy in descending priority
 *    pi(v) = splitmix64_finalizer((seed << 32) ^ v); self-loops ignored.
 *  - balanced coloring (optional; Sec. 6.2 leaves class-size balance to
 *    future work): the greedy colouring's over-full classes hand vertices to
 *    under-full ones, as defined at balance_colors below.
 *  - schedule (Sec. 6.1): colored phases while the phase graph has at least
 *    `color_cutoff` vertices and the phase-to-phase net gain stays at or
 *    above theta_color * |Q_prev|; then uncolored phases with theta_final until
 *    a phase gains less than that, does not shrink the graph, or the phase cap.
 *  - 2m = 0: every vertex alone, Q = 0 (numerator 0, denominator 1), no phase.
 */
#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <cstdio>
#include <map>
#include <set>
#include <utility>
#include <vector>

typedef __int128 i128;
typedef unsigned __int128 u128;

namespace {

struct Graph {
    int64_t n = 0;
    std::vector<int64_t> off;   // n+1
    std::vector<int32_t> col;   // nnz
    std::vector<int64_t> w;     // nnz
    int64_t nnz() const { return (int64_t)col.size(); }
};

Graph make_graph(int64_t n, const int64_t *off, const int32_t *col, const int32_t *w32,
                 const int64_t *w64)
{
    Graph g;
    g.n = n;
    g.off.assign(off, off + n + 1);
    int64_t nnz = off[n];
    g.col.assign(col, col + nnz);
    g.w.resize(nnz);
    for (int64_t e = 0; e < nnz; ++e) g.w[e] = w64 ? w64[e] : (w32 ? (int64_t)w32[e] : 1);
    return g;
}

/* 0 = valid; 1 = offsets; 2 = column out of range; 3 = columns not strictly
 * ascending; 4 = weight < 1; 5 = not symmetric (missing or different mirror) */
int validate(const Graph &g)
{
    if (g.off.size() != (size_t)g.n + 1 || g.off[0] != 0) return 1;
    for (int64_t i = 0; i < g.n; ++i)
        if (g.off[i + 1] < g.off[i]) return 1;
    if (g.off[g.n] != g.nnz()) return 1;
    for (int64_t i = 0; i < g.n; ++i)
        for (int64_t e = g.off[i]; e < g.off[i + 1]; ++e) {
            if (g.col[e] < 0 || g.col[e] >= g.n) return 2;
            if (e > g.off[i] && g.col[e] <= g.col[e - 1]) return 3;
            if (g.w[e] < 1) return 4;
        }
    for (int64_t i = 0; i < g.n; ++i)
        for (int64_t e = g.off[i]; e < g.off[i + 1]; ++e) {
            int32_t j = g.col[e];
            auto first = g.col.begin() + g.off[j], last = g.col.begin() + g.off[j + 1];
            auto it = std::lower_bound(first, last, (int32_t)i);   /* rows are sorted (checked above) */
            if (it == last || *it != i || g.w[it - g.col.begin()] != g.w[e]) return 5;
        }
    return 0;
}

/* weighted degrees k_i = sum of the row (Sec. 2), and 2m = sum_i k_i */
void degrees(const Graph &g, std::vector<int64_t> &k, int64_t &two_m)
{
    k.assign(g.n, 0);
    two_m = 0;
    for (int64_t i = 0; i < g.n; ++i) {
        for (int64_t e = g.off[i]; e < g.off[i + 1]; ++e) k[i] += g.w[e];
        two_m += k[i];
    }
}

/* Eq. 3 scaled by (2m)^2: N = 2m * sum_i e_{i->C(i)} - sum_C a_C^2, D = (2m)^2 */
void modularity(const Graph &g, const std::vector<int32_t> &C, i128 &N, i128 &D)
{
    std::vector<int64_t> k;
    int64_t two_m;
    degrees(g, k, two_m);
    if (two_m == 0) { N = 0; D = 1; return; }
    int64_t inside = 0;
    for (int64_t u = 0; u < g.n; ++u)
        for (int64_t e = g.off[u]; e < g.off[u + 1]; ++e)
            if (C[u] == C[g.col[e]]) inside += g.w[e];
    std::map<int32_t, int64_t> a;                       // Eq. 2
    for (int64_t u = 0; u < g.n; ++u) a[C[u]] += k[u];
    i128 sq = 0;
    for (const auto &kv : a) sq += (i128)kv.second * kv.second;
    N = (i128)two_m * inside - sq;
    D = (i128)two_m * two_m;
}

/* distinct labels in ascending order get dense new ids 0..K-1 */
int64_t renumber(const std::vector<int32_t> &C, std::vector<int32_t> &new_of)
{
    std::set<int32_t> used(C.begin(), C.end());
    new_of.assign(C.size(), -1);
    int32_t next = 0;
    for (int32_t c : used) new_of[c] = next++;
    return next;
}

/* community graph: W'(new C(u), new C(v)) = sum over entries (u,v,w) of w */
Graph coarsen(const Graph &g, const std::vector<int32_t> &C, std::vector<int32_t> &new_of)
{
    int64_t K = renumber(C, new_of);
    std::map<std::pair<int32_t, int32_t>, int64_t> W;
    for (int64_t u = 0; u < g.n; ++u)
        for (int64_t e = g.off[u]; e < g.off[u + 1]; ++e)
            W[{new_of[C[u]], new_of[C[g.col[e]]]}] += g.w[e];
    Graph h;
    h.n = K;
    h.off.assign(K + 1, 0);
    for (const auto &kv : W) {
        h.off[kv.first.first + 1]++;
        h.col.push_back(kv.first.second);
        h.w.push_back(kv.second);
    }
    for (int64_t c = 0; c < K; ++c) h.off[c + 1] += h.off[c];
    return h;
}

/* vertex following (Sec. 5.3): representative of each vertex */
std::vector<int32_t> vf_map(const Graph &g)
{
    std::vector<char> single(g.n, 0);
    for (int64_t i = 0; i < g.n; ++i)
        single[i] = (g.off[i + 1] - g.off[i] == 1) && (g.col[g.off[i]] != i);
    std::vector<int32_t> map(g.n);
    for (int64_t i = 0; i < g.n; ++i) {
        map[i] = (int32_t)i;
        if (!single[i]) continue;
        int32_t j = g.col[g.off[i]];
        map[i] = single[j] ? std::min<int32_t>((int32_t)i, j) : j;
    }
    return map;
}

/* one round of chain-compressing vertex following: i qualifies when its row
 * holds exactly one neighbour j != i (besides an optional self-loop) and
 * 2m * w_ij > k_i * k_j; it then merges into j, or, when j qualifies too
 * (the two only see each other), both go to the smaller id */
std::vector<int32_t> vf_chain_map(const Graph &g, const std::vector<int64_t> &k, int64_t two_m)
{
    std::vector<char> single(g.n, 0);
    std::vector<int32_t> nbr(g.n, -1);
    for (int64_t i = 0; i < g.n; ++i) {
        int64_t others = 0, w = 0;
        for (int64_t e = g.off[i]; e < g.off[i + 1]; ++e)
            if (g.col[e] != i) { ++others; nbr[i] = g.col[e]; w = g.w[e]; }
        single[i] = others == 1 && (i128)two_m * w > (i128)k[i] * k[nbr[i]];
    }
    std::vector<int32_t> map(g.n);
    for (int64_t i = 0; i < g.n; ++i) {
        map[i] = (int32_t)i;
        if (!single[i]) continue;
        const int32_t to = nbr[i];
        map[i] = single[to] ? std::min<int32_t>((int32_t)i, to) : to;
    }
    return map;
}

/* SplitMix64 output finalizer (Steele, Lea, Flood, OOPSLA 2014) */
uint64_t splitmix64_finalizer(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t priority(uint64_t seed, int64_t v) { return splitmix64_finalizer((seed << 32) ^ (uint64_t)v); }

/* greedy distance-1 coloring in descending priority order */
int32_t color_greedy(const Graph &g, uint64_t seed, std::vector<int32_t> &color)
{
    std::vector<int32_t> order(g.n);
    for (int64_t v = 0; v < g.n; ++v) order[v] = (int32_t)v;
    std::sort(order.begin(), order.end(),
              [&](int32_t x, int32_t y) { return priority(seed, x) > priority(seed, y); });
    color.assign(g.n, -1);
    int32_t ncolors = 0;
    for (int32_t v : order) {
        std::set<int32_t> taken;
        for (int64_t e = g.off[v]; e < g.off[v + 1]; ++e)
            if (g.col[e] != v && color[g.col[e]] >= 0) taken.insert(color[g.col[e]]);
        int32_t c = 0;
        while (taken.count(c)) ++c;
        color[v] = c;
        ncolors = std::max(ncolors, c + 1);
    }
    return ncolors;
}

/* Balanced colouring: equalises the class sizes of a proper colouring with
 * chi colours on n vertices towards gamma = ceil(n / chi), keeping it proper
 * and using no new colour.  The over-full classes (more than gamma vertices)
 * are taken one after another in ascending colour c.  A vertex v of K_c may
 * go to any colour c' != c that none of its neighbours has (self-loops
 * ignored) and whose class holds fewer than gamma vertices.  K_c is an
 * independent set, so these permissions do not change while K_c is handled.
 * Moves happen in rounds: every vertex of K_c still waiting proposes its
 * smallest admissible colour (a vertex with none stops waiting); the
 * proposers of each c' are taken in descending priority, at most
 * gamma - |K_c'| of them; of all the vertices taken, the first |K_c| - gamma
 * in descending priority move.  K_c is done when it is down to gamma or a
 * round moves nobody.  Returns the number of vertices moved. */
int64_t balance_colors(const Graph &g, uint64_t seed, std::vector<int32_t> &color, int32_t ncolors)
{
    if (g.n == 0 || ncolors == 0) return 0;
    const int64_t gamma = (g.n + ncolors - 1) / ncolors;
    std::vector<int64_t> size(ncolors, 0);
    for (int64_t v = 0; v < g.n; ++v) size[color[v]]++;
    std::vector<int32_t> order(g.n);
    for (int64_t v = 0; v < g.n; ++v) order[v] = (int32_t)v;
    std::sort(order.begin(), order.end(),
              [&](int32_t x, int32_t y) { return priority(seed, x) > priority(seed, y); });
    int64_t moved_total = 0;
    for (int32_t c = 0; c < ncolors; ++c) {
        if (size[c] <= gamma) continue;
        std::vector<int32_t> waiting;                    /* K_c in descending priority */
        for (int32_t v : order)
            if (color[v] == c) waiting.push_back(v);
        std::map<int32_t, std::set<int32_t>> used;       /* colours of each vertex's neighbours */
        for (int32_t v : waiting)
            for (int64_t e = g.off[v]; e < g.off[v + 1]; ++e)
                if (g.col[e] != v) used[v].insert(color[g.col[e]]);
        while (size[c] > gamma) {
            std::vector<int32_t> still, taken;
            std::map<int32_t, int32_t> proposal;
            std::map<int32_t, int64_t> count;
            for (int32_t v : waiting) {
                int32_t to = -1;
                for (int32_t d = 0; d < ncolors && to < 0; ++d)
                    if (d != c && size[d] < gamma && !used[v].count(d)) to = d;
                if (to < 0) continue;                    /* nothing admissible: stops waiting */
                still.push_back(v);
                proposal[v] = to;
                if (count[to] < gamma - size[to]) { taken.push_back(v); count[to]++; }
            }
            const int64_t room = size[c] - gamma;
            int64_t moved = 0;
            std::set<int32_t> gone;
            for (int32_t v : taken) {
                if (moved == room) break;
                size[c]--;
                size[proposal[v]]++;
                color[v] = proposal[v];
                gone.insert(v);
                ++moved;
            }
            if (moved == 0) break;
            moved_total += moved;
            waiting.clear();
            for (int32_t v : still)
                if (!gone.count(v)) waiting.push_back(v);
        }
    }
    return moved_total;
}

/* |x| for i128 as unsigned */
u128 uabs(i128 x) { return x < 0 ? (u128)(-(x + 1)) + 1 : (u128)x; }

/* exact compare of x*p < y*q for x, y < 2^127 and p, q < 2^64 (192-bit products) */
bool mul_less(u128 x, uint64_t p, u128 y, uint64_t q)
{
    auto wide = [](u128 a, uint64_t b, u128 &hi, uint64_t &lo) {
        u128 a0 = (uint64_t)a, a1 = a >> 64;
        u128 p0 = a0 * b, p1 = a1 * b;
        lo = (uint64_t)p0;
        hi = p1 + (p0 >> 64);
    };
    u128 h1, h2;
    uint64_t l1, l2;
    wide(x, p, h1, l1);
    wide(y, q, h2, l2);
    return h1 < h2 || (h1 == h2 && l1 < l2);
}

/* correctly rounded (round-half-even) double of N / D, D > 0, |N| <= D */
double ratio_to_double(i128 N, i128 D)
{
    if (N == 0) return 0.0;
    bool neg = N < 0;
    u128 r = uabs(N), d = (u128)D;
    /* integer part (0 or 1) then fraction bits by long division */
    uint64_t mant = 0;
    int bits = 0, exp = 0;  // value = mant * 2^(exp)
    bool started = false;
    if (r >= d) { mant = 1; bits = 1; r -= d; started = true; }
    int pos = 0;            // number of fraction bits produced
    while (bits < 54) {
        r <<= 1;
        ++pos;
        uint64_t b = (r >= d) ? 1 : 0;
        if (b) r -= d;
        if (started || b) {
            mant = (mant << 1) | b;
            ++bits;
            started = true;
        }
    }
    exp = -pos;
    /* mant has 54 bits: 53 kept + 1 round bit; sticky = remainder != 0 */
    uint64_t round_bit = mant & 1;
    mant >>= 1;
    exp += 1;
    bool sticky = (r != 0);
    if (round_bit && (sticky || (mant & 1))) {
        mant += 1;
        if (mant == (1ull << 53)) { mant >>= 1; exp += 1; }
    }
    double q = (double)mant;
    /* scale by 2^exp exactly */
    while (exp > 0) { q *= 2.0; --exp; }
    while (exp < 0) {
        int s = exp < -60 ? 60 : -exp;
        q /= (double)(1ull << s);
        exp += s;
    }
    return neg ? -q : q;
}

struct Params {
    int32_t vf = 0, color = 0, singlet_rule = 1, threshold_mode = 0, color_first_phase_only = 0, color_balance = 0;
    int64_t theta_color_num = 1, theta_color_den = 100;
    int64_t theta_final_num = 1, theta_final_den = 1000000;
    int64_t color_cutoff = 100000;
    int32_t max_iter = 1000, max_phases = 100;
    uint64_t color_seed = 0x4C4F5556ull;
};

/* net gain now - before below theta = num/den, relative to |before| (mode 0)
 * or absolute, i.e. relative to D (mode 1); any loss is below */
bool gain_below(i128 now, i128 before, i128 D, int64_t num, int64_t den, int mode)
{
    if (now < before) return true;
    u128 gain = (u128)(now - before);
    u128 ref = mode == 0 ? uabs(before) : (u128)D;
    return mul_less(gain, (uint64_t)den, ref, (uint64_t)num);
}

/* the evolving state of one phase on one graph */
struct State {
    Graph g;
    std::vector<int64_t> k;
    int64_t two_m = 0;
    std::vector<int32_t> C;      // community of each vertex
    std::vector<int64_t> a;      // community degree a_c (Eq. 2), indexed by id
    std::vector<int32_t> size;   // members per community
    std::vector<int32_t> color;  // empty = uncolored
    int32_t ncolors = 0;
    std::vector<int32_t> orig_map;
    int64_t n_orig = 0;

    void reset_singletons()
    {
        degrees(g, k, two_m);
        C.resize(g.n);
        a.assign(g.n, 0);
        size.assign(g.n, 0);
        for (int64_t i = 0; i < g.n; ++i) { C[i] = (int32_t)i; a[i] = k[i]; size[i] = 1; }
        color.clear();
        ncolors = 0;
    }

    /* G(c) for candidate c != C(i) and G_stay; e computed on the fly */
    void neighbour_weights(int64_t i, std::map<int32_t, int64_t> &e) const
    {
        e.clear();
        for (int64_t f = g.off[i]; f < g.off[i + 1]; ++f)
            if (g.col[f] != i) e[C[g.col[f]]] += g.w[f];                 // Eq. 1
    }
    i128 gain_to(int64_t i, int32_t c, int64_t e_ic) const
    {
        return (i128)two_m * e_ic - (i128)k[i] * a[c];
    }
    i128 gain_stay(int64_t i, int64_t e_iA) const
    {
        int32_t A = C[i];
        return (i128)two_m * e_iA - (i128)k[i] * (a[A] - k[i]);
    }

    /* decision for vertex i against the current state (Alg. 1 inner loop) */
    int32_t decide(int64_t i, int singlet_rule) const
    {
        std::map<int32_t, int64_t> e;
        neighbour_weights(i, e);
        int32_t A = C[i];
        int64_t eA = e.count(A) ? e.at(A) : 0;
        i128 stay = gain_stay(i, eA);
        bool have = false;
        i128 best = 0;
        int32_t best_c = A;
        for (const auto &kv : e) {              // ascending community id
            if (kv.first == A) continue;
            i128 G = gain_to(i, kv.first, kv.second);
            if (!have || G > best) { best = G; best_c = kv.first; have = true; }
        }
        if (!have || !(best > stay)) return A;
        if (singlet_rule && size[A] == 1 && size[best_c] == 1 && best_c > A) return A;
        return best_c;
    }

    void check_totals() const
    {
        std::vector<int64_t> a2(g.n, 0);
        std::vector<int32_t> s2(g.n, 0);
        int64_t tot = 0;
        for (int64_t i = 0; i < g.n; ++i) { a2[C[i]] += k[i]; s2[C[i]] += 1; }
        for (int64_t c = 0; c < g.n; ++c) tot += a2[c];
        if (a2 != a || s2 != size || tot != two_m) {
            fprintf(stderr, "oracle: community totals inconsistent\n");
            abort();
        }
    }

    /* one iteration; returns the number of vertices whose community changed */
    int64_t iterate(int singlet_rule)
    {
        std::vector<int32_t> start = C;
        std::vector<std::vector<int32_t>> classes;
        if (color.empty()) {
            classes.resize(1);
            for (int64_t i = 0; i < g.n; ++i) classes[0].push_back((int32_t)i);
        } else {
            classes.resize(ncolors);
            for (int64_t i = 0; i < g.n; ++i) classes[color[i]].push_back((int32_t)i);
        }
        for (const auto &K : classes) {
            std::vector<int32_t> next(K.size());
            for (size_t t = 0; t < K.size(); ++t) next[t] = decide(K[t], singlet_rule);
            for (size_t t = 0; t < K.size(); ++t) {
                int32_t i = K[t], A = C[i], B = next[t];
                if (A == B) continue;
                a[A] -= k[i]; a[B] += k[i];
                size[A] -= 1; size[B] += 1;
                C[i] = B;
            }
        }
        check_totals();
        int64_t moves = 0;
        for (int64_t i = 0; i < g.n; ++i) moves += (C[i] != start[i]);
        return moves;
    }

    /* replace the graph by its community graph; compose the vertex map */
    void coarsen_step()
    {
        std::vector<int32_t> new_of;
        Graph h = coarsen(g, C, new_of);
        for (int64_t x = 0; x < n_orig; ++x) orig_map[x] = new_of[C[orig_map[x]]];
        g = std::move(h);
        reset_singletons();
    }

    void vf_step()
    {
        std::vector<int32_t> m = vf_map(g);
        C = m;
        coarsen_step();
    }

    /* chain compression: rounds until no vertex qualifies; returns the rounds that merged */
    int64_t vf_chain_step()
    {
        int64_t rounds = 0;
        for (;;) {
            std::vector<int32_t> m = vf_chain_map(g, k, two_m);
            bool any = false;
            for (int64_t i = 0; i < g.n && !any; ++i) any = m[i] != i;
            if (!any) return rounds;
            C = m;
            coarsen_step();
            ++rounds;
        }
    }
};

struct PhaseRec {
    int64_t n, nnz, colored, ncolors, iterations, hit_max_iter, first_iter;
    i128 N_end;
    int64_t undone;   /* the last iteration lost modularity and was undone */
};
struct IterRec { int64_t moves; i128 N; };

struct Result {
    int64_t n_orig = 0, K = 0, n_vf = 0, vf_rounds = 0;
    i128 N = 0, D = 1, N0 = 0;
    double q = 0.0;
    std::vector<int32_t> labels;
    std::vector<PhaseRec> phases;
    std::vector<IterRec> iters;
    std::vector<std::vector<int32_t>> phase_labels; /* composed labels after each phase */
};

void run(const Graph &input, const Params &P, Result &R)
{
    State st;
    st.g = input;
    st.n_orig = input.n;
    st.orig_map.resize(input.n);
    for (int64_t x = 0; x < input.n; ++x) st.orig_map[x] = (int32_t)x;
    st.reset_singletons();
    R = Result();
    R.n_orig = input.n;
    if (st.two_m == 0) {
        R.labels = st.orig_map;
        R.K = input.n;
        R.n_vf = input.n;
        return;
    }
    const i128 D = (i128)st.two_m * st.two_m;
    if (P.vf == 1) st.vf_step();
    if (P.vf == 2) R.vf_rounds = st.vf_chain_step();
    R.n_vf = st.g.n;
    i128 N, Dd;
    modularity(st.g, st.C, N, Dd);
    R.N0 = N;
    i128 Q_prev = N;
    bool still_coloring = P.color != 0;
    for (int64_t p = 1;; ++p) {
        bool colored = still_coloring && st.g.n >= P.color_cutoff;
        int64_t tnum = colored ? P.theta_color_num : P.theta_final_num;
        int64_t tden = colored ? P.theta_color_den : P.theta_final_den;
        if (colored) {
            st.ncolors = color_greedy(st.g, P.color_seed, st.color);
            if (P.color_balance) balance_colors(st.g, P.color_seed, st.color, st.ncolors);
        }
        PhaseRec ph{};
        ph.n = st.g.n;
        ph.nnz = st.g.nnz();
        ph.colored = colored;
        ph.ncolors = colored ? st.ncolors : 0;
        ph.first_iter = (int64_t)R.iters.size();
        i128 N_prev = Q_prev, N_t = Q_prev;   /* the phase starts from singletons of G_p */
        int64_t t = 0;
        for (;;) {
            ++t;
            const std::vector<int32_t> C_before = st.C;
            int64_t moves = st.iterate(P.singlet_rule);
            modularity(st.g, st.C, N_t, Dd);
            R.iters.push_back({moves, N_t});
            if (moves == 0) break;
            if (N_t < N_prev) {                     /* a loss: back to the partition before it */
                st.C = C_before;
                std::fill(st.a.begin(), st.a.end(), 0);
                std::fill(st.size.begin(), st.size.end(), 0);
                for (int64_t i = 0; i < st.g.n; ++i) { st.a[st.C[i]] += st.k[i]; st.size[st.C[i]] += 1; }
                N_t = N_prev;
                ph.undone = 1;
                break;
            }
            if (t >= 2 && gain_below(N_t, N_prev, D, tnum, tden, P.threshold_mode)) break;
            if (t >= P.max_iter) { ph.hit_max_iter = 1; break; }
            N_prev = N_t;
        }
        ph.iterations = t;
        ph.N_end = N_t;
        R.phases.push_back(ph);
        int64_t n_before = st.g.n;
        st.coarsen_step();
        R.phase_labels.push_back(st.orig_map);
        int64_t n_after = st.g.n;
        bool stop;
        if (colored) {
            if (n_after < P.color_cutoff || n_after == n_before || P.color_first_phase_only ||
                gain_below(N_t, Q_prev, D, P.theta_color_num, P.theta_color_den, 0))
                still_coloring = false;
            stop = (p >= P.max_phases);
        } else {
            stop = (n_after == n_before) || (p >= P.max_phases) ||
                   gain_below(N_t, Q_prev, D, P.theta_final_num, P.theta_final_den, 0);
        }
        Q_prev = N_t;
        if (stop) break;
    }
    R.labels = st.orig_map;
    R.K = st.g.n;
    R.N = Q_prev;
    R.D = D;
    R.q = ratio_to_double(R.N, R.D);
}

void put128(i128 v, int64_t *out) { out[0] = (int64_t)(uint64_t)(u128)v; out[1] = (int64_t)(v >> 64); }

Params params_from(const int64_t *p)
{
    /* flat parameter vector: vf, color, singlet_rule, threshold_mode,
     * color_first_phase_only, tc_num, tc_den, tf_num, tf_den, cutoff,
     * max_iter, max_phases, seed, color_balance */
    Params P;
    P.vf = (int32_t)p[0]; P.color = (int32_t)p[1]; P.singlet_rule = (int32_t)p[2];
    P.threshold_mode = (int32_t)p[3]; P.color_first_phase_only = (int32_t)p[4];
    P.theta_color_num = p[5]; P.theta_color_den = p[6];
    P.theta_final_num = p[7]; P.theta_final_den = p[8];
    P.color_cutoff = p[9]; P.max_iter = (int32_t)p[10]; P.max_phases = (int32_t)p[11];
    P.color_seed = (uint64_t)p[12];
    P.color_balance = (int32_t)p[13];
    return P;
}

} // namespace

/* ====================================================================== */
/* C interface (ctypes)                                                   */
/* ====================================================================== */
extern "C" {

int oracle_validate(int64_t n, const int64_t *off, const int32_t *col, const int32_t *w32)
{
    for (int64_t i = 0; i < n; ++i)
        if (off[i + 1] < off[i]) return 1;
    if (off[0] != 0) return 1;
    Graph g = make_graph(n, off, col, w32, nullptr);
    return validate(g);
}

void oracle_degrees(int64_t n, const int64_t *off, const int32_t *col, const int32_t *w32,
                    int64_t *k_out, int64_t *two_m_out)
{
    Graph g = make_graph(n, off, col, w32, nullptr);
    std::vector<int64_t> k;
    degrees(g, k, *two_m_out);
    std::copy(k.begin(), k.end(), k_out);
}

void oracle_modularity(int64_t n, const int64_t *off, const int32_t *col, const int32_t *w32,
                       const int64_t *w64, const int32_t *labels, int64_t *N_out, int64_t *D_out)
{
    Graph g = make_graph(n, off, col, w32, w64);
    std::vector<int32_t> C(labels, labels + n);
    i128 N, D;
    modularity(g, C, N, D);
    put128(N, N_out);
    put128(D, D_out);
}

uint64_t oracle_mix64(uint64_t z) { return splitmix64_finalizer(z); }

double oracle_ratio_to_double(int64_t nlo, int64_t nhi, int64_t dlo, int64_t dhi)
{
    i128 N = ((i128)nhi << 64) | (u128)(uint64_t)nlo;
    i128 D = ((i128)dhi << 64) | (u128)(uint64_t)dlo;
    return ratio_to_double(N, D);
}

/* ---- step-wise state ---- */
void *oracle_state_new(int64_t n, const int64_t *off, const int32_t *col, const int32_t *w32)
{
    State *st = new State();
    st->g = make_graph(n, off, col, w32, nullptr);
    st->n_orig = n;
    st->orig_map.resize(n);
    for (int64_t x = 0; x < n; ++x) st->orig_map[x] = (int32_t)x;
    st->reset_singletons();
    return st;
}

void oracle_state_free(void *h) { delete (State *)h; }

/* out: n, nnz, 2m, ncolors, n_orig */
void oracle_state_info(void *h, int64_t *out)
{
    State *st = (State *)h;
    out[0] = st->g.n; out[1] = st->g.nnz(); out[2] = st->two_m; out[3] = st->ncolors; out[4] = st->n_orig;
}

void oracle_state_vf(void *h) { ((State *)h)->vf_step(); }

/* chain-compressing vertex following; returns the rounds that merged */
int64_t oracle_state_vf_chain(void *h) { return ((State *)h)->vf_chain_step(); }

int32_t oracle_state_color(void *h, uint64_t seed)
{
    State *st = (State *)h;
    st->ncolors = color_greedy(st->g, seed, st->color);
    return st->ncolors;
}

/* balanced colouring of the current colouring; returns the vertices moved */
int64_t oracle_state_balance(void *h, uint64_t seed)
{
    State *st = (State *)h;
    return balance_colors(st->g, seed, st->color, st->ncolors);
}

void oracle_state_uncolor(void *h)
{
    State *st = (State *)h;
    st->color.clear();
    st->ncolors = 0;
}

/* one iteration: returns moves; N_out = modularity numerator of the new state */
int64_t oracle_state_iterate(void *h, int32_t singlet_rule, int64_t *N_out)
{
    State *st = (State *)h;
    int64_t moves = st->iterate(singlet_rule);
    i128 N, D;
    modularity(st->g, st->C, N, D);
    put128(N, N_out);
    return moves;
}

int64_t oracle_state_coarsen(void *h)
{
    State *st = (State *)h;
    st->coarsen_step();
    return st->g.n;
}

/* which: 0 comm int32[n], 1 a int64[n], 2 size int32[n], 3 k int64[n],
 * 4 color int32[n], 5 offsets int64[n+1], 6 cols int32[nnz],
 * 7 weights int64[nnz], 8 orig_map int32[n_orig] */
void oracle_state_get(void *h, int32_t which, void *out)
{
    State *st = (State *)h;
    switch (which) {
    case 0: std::copy(st->C.begin(), st->C.end(), (int32_t *)out); break;
    case 1: std::copy(st->a.begin(), st->a.end(), (int64_t *)out); break;
    case 2: std::copy(st->size.begin(), st->size.end(), (int32_t *)out); break;
    case 3: std::copy(st->k.begin(), st->k.end(), (int64_t *)out); break;
    case 4: std::copy(st->color.begin(), st->color.end(), (int32_t *)out); break;
    case 5: std::copy(st->g.off.begin(), st->g.off.end(), (int64_t *)out); break;
    case 6: std::copy(st->g.col.begin(), st->g.col.end(), (int32_t *)out); break;
    case 7: std::copy(st->g.w.begin(), st->g.w.end(), (int64_t *)out); break;
    case 8: std::copy(st->orig_map.begin(), st->orig_map.end(), (int32_t *)out); break;
    default: break;
    }
}

/* set the community assignment (a and size recomputed from scratch) */
void oracle_state_set_comm(void *h, const int32_t *comm)
{
    State *st = (State *)h;
    for (int64_t i = 0; i < st->g.n; ++i) st->C[i] = comm[i];
    std::fill(st->a.begin(), st->a.end(), 0);
    std::fill(st->size.begin(), st->size.end(), 0);
    for (int64_t i = 0; i < st->g.n; ++i) { st->a[st->C[i]] += st->k[i]; st->size[st->C[i]] += 1; }
}

/* gains of vertex i: G(c) for a candidate c (e computed from the row) and G_stay */
void oracle_state_gain(void *h, int64_t i, int32_t c, int64_t *G_out, int64_t *stay_out)
{
    State *st = (State *)h;
    std::map<int32_t, int64_t> e;
    st->neighbour_weights(i, e);
    int64_t eic = e.count(c) ? e.at(c) : 0;
    int64_t eA = e.count(st->C[i]) ? e.at(st->C[i]) : 0;
    put128(st->gain_to(i, c, eic), G_out);
    put128(st->gain_stay(i, eA), stay_out);
}

int32_t oracle_state_decide(void *h, int64_t i, int32_t singlet_rule)
{
    return ((State *)h)->decide(i, singlet_rule);
}

/* decisions of vertices [lo, hi) against the current state (nothing applied);
 * returns the number of CSR entries those rows hold */
int64_t oracle_state_decide_range(void *h, int64_t lo, int64_t hi, int32_t singlet_rule, int32_t *out)
{
    State *st = (State *)h;
    for (int64_t i = lo; i < hi; ++i) out[i - lo] = st->decide(i, singlet_rule);
    return st->g.off[hi] - st->g.off[lo];
}

/* ---- full run ---- */
void *oracle_run(int64_t n, const int64_t *off, const int32_t *col, const int32_t *w32,
                 const int64_t *params)
{
    Graph g = make_graph(n, off, col, w32, nullptr);
    Result *R = new Result();
    run(g, params_from(params), *R);
    return R;
}

void oracle_result_free(void *h) { delete (Result *)h; }

/* out: n_orig, K, n_vf, phases, iterations, N(lo,hi), D(lo,hi), N0(lo,hi), vf_rounds */
void oracle_result_scalars(void *h, int64_t *out, double *q)
{
    Result *R = (Result *)h;
    out[0] = R->n_orig; out[1] = R->K; out[2] = R->n_vf;
    out[3] = (int64_t)R->phases.size(); out[4] = (int64_t)R->iters.size();
    put128(R->N, out + 5);
    put128(R->D, out + 7);
    put128(R->N0, out + 9);
    out[11] = R->vf_rounds;
    *q = R->q;
}

void oracle_result_labels(void *h, int32_t *out)
{
    Result *R = (Result *)h;
    std::copy(R->labels.begin(), R->labels.end(), out);
}

void oracle_result_phase_labels(void *h, int64_t p, int32_t *out)
{
    Result *R = (Result *)h;
    std::copy(R->phase_labels[p].begin(), R->phase_labels[p].end(), out);
}

/* out: n, nnz, colored, ncolors, iterations, hit_max_iter, first_iter, N_end(lo,hi), undone */
void oracle_result_phase(void *h, int64_t p, int64_t *out)
{
    const PhaseRec &ph = ((Result *)h)->phases[p];
    out[0] = ph.n; out[1] = ph.nnz; out[2] = ph.colored; out[3] = ph.ncolors;
    out[4] = ph.iterations; out[5] = ph.hit_max_iter; out[6] = ph.first_iter;
    put128(ph.N_end, out + 7);
    out[9] = ph.undone;
}

/* out: moves, N(lo,hi) */
void oracle_result_iter(void *h, int64_t t, int64_t *out)
{
    const IterRec &it = ((Result *)h)->iters[t];
    out[0] = it.moves;
    put128(it.N, out + 1);
}

} // extern "C"
