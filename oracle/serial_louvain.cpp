/*
 * SERIAL LOUVAIN -- test and baseline infrastructure only (a CPU comparison
 * system, never part of the GPU library).
 *
 * The original, sequential Louvain method as the paper recounts it in Sec. 3
 * (Blondel et al.): within an iteration the vertices are visited one after
 * the other in a fixed order (ascending id), and each vertex's move is
 * applied at once, so the next vertex already sees it (the "latest
 * information" of Sec. 4); iterations repeat until the net gain is
 * negligible, then the graph is collapsed into one vertex per community and
 * the next phase starts.  The paper compares its parallel heuristics against
 * this method for modularity (Table 2) and for the composition of the
 * communities (Table 3).
 *
 * Exact integer arithmetic throughout, with the same conventions as the
 * synchronous oracle: self-loops stored once and counted once in k_i and in
 * the internal weight; for vertex i in community A and candidate c != A,
 * 2m^2 * dQ = G(c) - G_stay with G(c) = 2m*e_{i->c} - k_i*a_c and
 * G_stay = 2m*e_{i->A\{i}} - k_i*(a_A - k_i) (Eq. 4); the target is the
 * lexicographic max of (G(c), -c) and the vertex moves iff G(c*) > G_stay.
 * Because each move is taken against the current state, every move raises
 * Q, so an iteration never loses modularity.  Iteration stop: nothing moved,
 * or from the second iteration on a gain below theta * |Q_{t-1}|; phase stop:
 * no shrink, a phase gain below theta * |Q_prev|, or the phase cap.
 * Communities are renumbered in ascending id after each phase.
 *
 * Data structures are the plainest available (std::map per vertex, std::map
 * keyed by community pairs for the rebuild); nothing is shared with the
 * synchronous oracle or the GPU library.
 */
#include <cstdint>
#include <map>
#include <set>
#include <utility>
#include <vector>

typedef __int128 s128;
typedef unsigned __int128 s128u;

namespace {

struct Csr {
    int64_t n = 0;
    std::vector<int64_t> off;
    std::vector<int32_t> col;
    std::vector<int64_t> w;
};

s128u magnitude(s128 x) { return x < 0 ? (s128u)0 - (s128u)x : (s128u)x; }

/* gain < theta * |before|, theta = num / den (exact: both sides scaled by den) */
bool small_gain(s128 now, s128 before, int64_t num, int64_t den)
{
    if (now < before) return true;
    /* gain * den and |before| * num can pass 2^127: compared as 192-bit
     * products (a 128-bit high part and a 64-bit low part) */
    s128u g = (s128u)(now - before), r = magnitude(before);
    auto mul = [](s128u a, uint64_t b, s128u &hi, uint64_t &lo) {
        s128u p0 = (s128u)(uint64_t)a * b, p1 = (s128u)(uint64_t)(a >> 64) * b;
        lo = (uint64_t)p0;
        hi = p1 + (p0 >> 64);
    };
    s128u h1, h2;
    uint64_t l1, l2;
    mul(g, (uint64_t)den, h1, l1);
    mul(r, (uint64_t)num, h2, l2);
    return h1 < h2 || (h1 == h2 && l1 < l2);
}

struct Phase {
    Csr g;
    std::vector<int64_t> k;
    int64_t two_m = 0;
    std::vector<int32_t> C;
    std::vector<int64_t> a;

    void start()
    {
        k.assign(g.n, 0);
        two_m = 0;
        for (int64_t i = 0; i < g.n; ++i) {
            for (int64_t e = g.off[i]; e < g.off[i + 1]; ++e) k[i] += g.w[e];
            two_m += k[i];
        }
        C.resize(g.n);
        a = k;
        for (int64_t i = 0; i < g.n; ++i) C[i] = (int32_t)i;
    }

    /* Eq. 3 scaled by (2m)^2 */
    s128 numerator() const
    {
        int64_t inside = 0;
        for (int64_t u = 0; u < g.n; ++u)
            for (int64_t e = g.off[u]; e < g.off[u + 1]; ++e)
                if (C[u] == C[g.col[e]]) inside += g.w[e];
        std::map<int32_t, int64_t> tot;
        for (int64_t u = 0; u < g.n; ++u) tot[C[u]] += k[u];
        s128 sq = 0;
        for (const auto &kv : tot) sq += (s128)kv.second * kv.second;
        return (s128)two_m * inside - sq;
    }

    /* one in-order pass with immediate updates; returns the moves */
    int64_t pass()
    {
        int64_t moves = 0;
        for (int64_t i = 0; i < g.n; ++i) {
            std::map<int32_t, int64_t> e;
            for (int64_t f = g.off[i]; f < g.off[i + 1]; ++f)
                if (g.col[f] != i) e[C[g.col[f]]] += g.w[f];
            const int32_t A = C[i];
            const int64_t eA = e.count(A) ? e[A] : 0;
            const s128 stay = (s128)two_m * eA - (s128)k[i] * (a[A] - k[i]);
            bool have = false;
            s128 best = 0;
            int32_t best_c = A;
            for (const auto &kv : e) {
                if (kv.first == A) continue;
                const s128 G = (s128)two_m * kv.second - (s128)k[i] * a[kv.first];
                if (!have || G > best) { best = G; best_c = kv.first; have = true; }
            }
            if (have && best > stay) {
                a[A] -= k[i];
                a[best_c] += k[i];
                C[i] = best_c;
                ++moves;
            }
        }
        return moves;
    }

    /* the community graph; new_of maps old community ids to dense new ids */
    Csr collapse(std::vector<int32_t> &new_of) const
    {
        std::set<int32_t> used(C.begin(), C.end());
        new_of.assign(g.n, -1);
        int32_t next = 0;
        for (int32_t c : used) new_of[c] = next++;
        std::map<std::pair<int32_t, int32_t>, int64_t> W;
        for (int64_t u = 0; u < g.n; ++u)
            for (int64_t f = g.off[u]; f < g.off[u + 1]; ++f)
                W[{new_of[C[u]], new_of[C[g.col[f]]]}] += g.w[f];
        Csr h;
        h.n = next;
        h.off.assign(next + 1, 0);
        for (const auto &kv : W) {
            h.off[kv.first.first + 1]++;
            h.col.push_back(kv.first.second);
            h.w.push_back(kv.second);
        }
        for (int64_t c = 0; c < next; ++c) h.off[c + 1] += h.off[c];
        return h;
    }
};

struct SerialResult {
    std::vector<int32_t> labels;
    int64_t K = 0, phases = 0, iterations = 0;
    s128 N = 0, D = 1;
};

void serial_louvain(const Csr &input, int64_t tnum, int64_t tden, int32_t max_iter, int32_t max_phases,
                    SerialResult &R)
{
    Phase ph;
    ph.g = input;
    ph.start();
    R = SerialResult();
    R.labels.resize(input.n);
    for (int64_t x = 0; x < input.n; ++x) R.labels[x] = (int32_t)x;
    R.K = input.n;
    if (ph.two_m == 0) return;
    R.D = (s128)ph.two_m * ph.two_m;
    s128 Q_prev = ph.numerator();
    for (int32_t p = 1;; ++p) {
        s128 N_prev = Q_prev, N_t = Q_prev;
        for (int32_t t = 1;; ++t) {
            const int64_t moves = ph.pass();
            ++R.iterations;
            N_t = ph.numerator();
            if (moves == 0) break;
            if (t >= 2 && small_gain(N_t, N_prev, tnum, tden)) break;
            if (t >= max_iter) break;
            N_prev = N_t;
        }
        ++R.phases;
        const int64_t n_before = ph.g.n;
        std::vector<int32_t> new_of;
        Csr h = ph.collapse(new_of);
        for (int64_t x = 0; x < input.n; ++x) R.labels[x] = new_of[ph.C[R.labels[x]]];
        ph.g = std::move(h);
        ph.start();
        const bool stop = ph.g.n == n_before || p >= max_phases || small_gain(N_t, Q_prev, tnum, tden);
        Q_prev = N_t;
        if (stop) break;
    }
    R.K = ph.g.n;
    R.N = Q_prev;
}

void put(s128 v, int64_t *out)
{
    out[0] = (int64_t)(uint64_t)(s128u)v;
    out[1] = (int64_t)(v >> 64);
}

} // namespace

extern "C" {

/* Runs the serial method on a symmetric CSR (weights NULL = unit).
 * out: K, phases, iterations, N(lo, hi), D(lo, hi); labels_out: n dense
 * labels in ascending order of community id. */
void serial_louvain_run(int64_t n, const int64_t *off, const int32_t *col, const int32_t *w, int64_t theta_num,
                        int64_t theta_den, int32_t max_iter, int32_t max_phases, int32_t *labels_out, int64_t *out)
{
    Csr g;
    g.n = n;
    g.off.assign(off, off + n + 1);
    g.col.assign(col, col + off[n]);
    g.w.resize(off[n]);
    for (int64_t e = 0; e < off[n]; ++e) g.w[e] = w ? w[e] : 1;
    SerialResult R;
    serial_louvain(g, theta_num, theta_den, max_iter, max_phases, R);
    for (int64_t x = 0; x < n; ++x) labels_out[x] = R.labels[x];
    out[0] = R.K;
    out[1] = R.phases;
    out[2] = R.iterations;
    put(R.N, out + 3);
    put(R.D, out + 5);
}

} // extern "C"
