"""Pins of the oracle to facts outside itself.

Each check takes an ``oracle.Oracle`` so that the same checks can be run on
deliberately broken copies of the oracle (test_oracle_mutants.py).

Independent references used here (none calls the oracle's arithmetic):
  * ``n_modmatrix``: modularity in the pairwise modularity-matrix form
    Q = (1/2m) sum_ij (A_ij - k_i k_j / 2m) [c_i == c_j] (Newman's form, which
    the paper's Eq. 3 rewrites per community), evaluated on the dense
    adjacency matrix, scaled by (2m)^2;
  * brute force over all set partitions for n <= 10;
  * closed forms for singletons, disjoint cliques and rings of cliques;
  * the published first output of SplitMix64 with seed 0;
  * Python's correctly rounded float(Fraction(N, D)).
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np

import small_graphs as SG


# ---------------------------------------------------------------------------
# independent evaluators
# ---------------------------------------------------------------------------
def dense(g):
    A = np.zeros((g.n, g.n), dtype=np.int64)
    rows = np.repeat(np.arange(g.n), np.diff(g.offsets))
    w = np.ones(g.nnz, dtype=np.int64) if g.weights is None else g.weights.astype(np.int64)
    A[rows, g.cols] = w
    return A


def dense_w64(n, off, cols, w):
    A = np.zeros((n, n), dtype=np.int64)
    rows = np.repeat(np.arange(n), np.diff(off))
    A[rows, cols] = w
    return A


def n_modmatrix_A(A, labels):
    """(N, D): N = sum_ij (2m A_ij - k_i k_j) [c_i == c_j], D = (2m)^2."""
    k = A.sum(axis=1)
    two_m = int(k.sum())
    if two_m == 0:
        return 0, 1
    lab = np.asarray(labels)
    same = lab[:, None] == lab[None, :]
    B = two_m * A - np.outer(k, k)
    return int(B[same].sum()), two_m * two_m


def n_modmatrix(g, labels):
    return n_modmatrix_A(dense(g), labels)


def set_partitions(n):
    """All set partitions of range(n) as restricted growth strings."""
    a = [0] * n

    def rec(i, m):
        if i == n:
            yield list(a)
            return
        for v in range(m + 2):
            a[i] = v
            yield from rec(i + 1, max(m, v))
    if n == 0:
        yield []
        return
    a[0] = 0
    yield from rec(1, 0)


def best_partition_N(g):
    A = dense(g)
    best = None
    for p in set_partitions(g.n):
        N, D = n_modmatrix_A(A, p)
        if best is None or N > best:
            best = N
    return best, D


def mix64_published_check(O):
    # SplitMix64 (Steele, Lea, Flood 2014) with seed 0: the state advances by the
    # golden gamma 0x9e3779b97f4a7c15 and the first output is 0xe220a8397b1dcdaf,
    # the second 0x6e789e6aa1b965f4.
    assert O.mix64(0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF
    assert O.mix64((2 * 0x9E3779B97F4A7C15) & ((1 << 64) - 1)) == 0x6E789E6AA1B965F4


# ---------------------------------------------------------------------------
# pins
# ---------------------------------------------------------------------------
def rand_graphs(seed=7, count=12):
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        n = int(rng.integers(4, 13))
        out.append(SG.random_graph(rng, n, p=float(rng.uniform(0.2, 0.6)),
                                   self_loops=0.3 if t % 2 else 0.0, wmax=1 if t % 3 == 0 else 9))
    return out


def p1_singleton_closed_form(O):
    """P1: singletons give Q0 = sum_i w_ii / 2m - sum_i k_i^2 / (2m)^2."""
    for g in rand_graphs(11):
        A = dense(g)
        k = A.sum(axis=1)
        two_m = int(k.sum())
        expect = two_m * int(np.trace(A)) - int((k * k).sum())
        N, D = O.modularity(g, np.arange(g.n))
        assert (N, D) == (expect, two_m * two_m)
        res = O.run(g)
        assert res.N0 == expect


def p2_totals_invariant(O):
    """P2: after every iteration (colored or not) sum a = 2m and sum size = n;
    and modularity of arbitrary partitions equals the modularity-matrix form."""
    rng = np.random.default_rng(3)
    for idx, g in enumerate(rand_graphs(12)):
        labels = rng.integers(0, max(1, g.n // 2), size=g.n)
        assert O.modularity(g, labels) == n_modmatrix(g, labels)
        st = O.state(g)
        if idx % 2:
            st.color()
        two_m = st.info()["two_m"]
        for _ in range(4):
            st.iterate(1)
            a, size = st.get("a"), st.get("size")
            comm = st.get("comm")
            assert int(a.sum()) == two_m and int(size.sum()) == g.n
            k = dense(g).sum(axis=1)
            for c in range(g.n):
                assert a[c] == int(k[comm == c].sum()) and size[c] == int((comm == c).sum())


def p3_single_move_is_eq4(O):
    """P3: for one move of i from A to c, N_after - N_before = 2 (G(c) - G_stay)
    (Eq. 4 scaled by 2 m^2, checked against the modularity-matrix form)."""
    rng = np.random.default_rng(5)
    for g in rand_graphs(21):
        st = O.state(g)
        for _ in range(6):
            comm = rng.integers(0, max(1, g.n // 2), size=g.n).astype(np.int32)
            st.set_comm(comm)
            i = int(rng.integers(0, g.n))
            nbrs = g.cols[g.offsets[i]:g.offsets[i + 1]]
            cands = sorted({int(comm[j]) for j in nbrs if j != i} - {int(comm[i])})
            if not cands:
                continue
            c = cands[int(rng.integers(0, len(cands)))]
            G, stay = st.gain(i, c)
            before, _ = n_modmatrix(g, comm)
            moved = comm.copy()
            moved[i] = c
            after, _ = n_modmatrix(g, moved)
            assert after - before == 2 * (G - stay)


def p4_eq6_two_moves(O):
    """P4 (Eq. 6): i and j moving into C(k) together change N by
    dN_i + dN_j + 4m w(i,j) - 2 k_i k_j."""
    rng = np.random.default_rng(9)
    checked = 0
    for g in rand_graphs(31, 20):
        A = dense(g)
        kdeg = A.sum(axis=1)
        two_m = int(kdeg.sum())
        st = O.state(g)
        for _ in range(10):
            if g.n < 3:
                break
            comm = np.arange(g.n, dtype=np.int32)
            i, j, k = (int(x) for x in rng.choice(g.n, 3, replace=False))
            st.set_comm(comm)
            target = int(comm[k])
            Gi, si = st.gain(i, target)
            Gj, sj = st.gain(j, target)
            before, _ = n_modmatrix(g, comm)
            both = comm.copy()
            both[i] = target
            both[j] = target
            after, _ = n_modmatrix(g, both)
            expect = 2 * (Gi - si) + 2 * (Gj - sj) + 2 * two_m * int(A[i, j]) - 2 * int(kdeg[i]) * int(kdeg[j])
            assert after - before == expect
            checked += 1
    assert checked > 50


def p5_lemma3(O):
    """P5 (Lemma 3): a degree-one vertex i with neighbour j outside its
    community always has G(C(j)) - G_stay > 0, and moves to C(j) unless the
    singlet rule vetoes."""
    rng = np.random.default_rng(13)
    checked = 0
    for t in range(30):
        n = int(rng.integers(5, 12))
        base = SG.random_graph(rng, n - 1, p=0.5, wmax=1 if t % 2 else 7)
        j = int(rng.integers(0, n - 1))
        edges, ws = [], []
        for u in range(n - 1):
            for e in range(base.offsets[u], base.offsets[u + 1]):
                v = int(base.cols[e])
                if u <= v:
                    edges.append((u, v))
                    ws.append(1 if base.weights is None else int(base.weights[e]))
        edges.append((n - 1, j))
        ws.append(int(rng.integers(1, 8)))
        g = SG.from_edges(n, edges, ws)
        st = O.state(g)
        for _ in range(5):
            comm = rng.integers(0, n, size=n).astype(np.int32)
            i = n - 1
            if comm[i] == comm[j]:
                comm[i] = (comm[j] + 1) % n
            st.set_comm(comm)
            G, stay = st.gain(i, int(comm[j]))
            assert G - stay > 0
            size = st.get("size")
            veto = size[comm[i]] == 1 and size[comm[j]] == 1 and comm[j] > comm[i]
            assert st.decide(i, 1) == (comm[i] if veto else comm[j])
            assert st.decide(i, 0) == comm[j]
            checked += 1
    assert checked == 150


def _check_csr(n, off, cols, w):
    assert off[0] == 0 and np.all(np.diff(off) >= 0) and off[-1] == len(cols)
    for i in range(n):
        r = cols[off[i]:off[i + 1]]
        assert np.all(np.diff(r) > 0)
    A = dense_w64(n, off, cols, w)
    assert np.array_equal(A, A.T)
    assert np.all(w >= 1)


def p6_coarsen_invariance(O):
    """P6: Q(G, C) = Q(G', singletons), 2m preserved, coarse CSR symmetric,
    sorted, unique; VF coarsening likewise."""
    rng = np.random.default_rng(17)
    for g in rand_graphs(41):
        for mode in range(3):
            st = O.state(g)
            if mode == 0:
                comm = rng.integers(0, max(1, g.n // 3), size=g.n).astype(np.int32)
                st.set_comm(comm)
            elif mode == 1:
                st.iterate(1)
                comm = st.get("comm")
            else:
                st.vf()
                comm = None
            two_m = st.info()["two_m"]
            if comm is not None:
                before = n_modmatrix(g, comm)
                st.coarsen()
            else:
                before = n_modmatrix(g, st.get("orig_map"))
            info = st.info()
            off, cols, w = st.get("offsets"), st.get("cols"), st.get("weights")
            _check_csr(info["n"], off, cols, w)
            A2 = dense_w64(info["n"], off, cols, w)
            assert int(A2.sum()) == two_m == info["two_m"]
            assert n_modmatrix_A(A2, np.arange(info["n"])) == before
            # composed map sends every original vertex to its coarse vertex
            om = st.get("orig_map")
            assert n_modmatrix(g, om) == before


def p7_phase_q_from_scratch(O):
    """P7: every phase's reported N equals the modularity-matrix Q of the
    composed labels on the original graph."""
    import oracle as OR
    for idx, g in enumerate(rand_graphs(51) + [SG.ring_of_cliques(5, 4)]):
        params = OR.Params(vf=idx % 2, color=idx % 3 == 0, color_cutoff=1)
        res = O.run(g, params, phase_labels=True)
        for ph, lab in zip(res.phases, res.phase_labels):
            assert n_modmatrix(g, lab) == (ph.N_end, res.D)
        assert n_modmatrix(g, res.labels) == (res.N, res.D)
        assert len(np.unique(res.labels)) == res.K
        assert np.array_equal(np.unique(res.labels), np.arange(res.K))


def p8_disjoint_cliques(O):
    """P8: r disjoint K_s are recovered exactly with Q = 1 - 1/r."""
    import oracle as OR
    rng = np.random.default_rng(19)
    for r, s in [(2, 3), (3, 4), (5, 5), (4, 7)]:
        perm = rng.permutation(r * s)
        g = SG.cliques(r, s, perm)
        for params in [OR.Params(), OR.Params(singlet_rule=0), OR.Params(vf=1, color=1, color_cutoff=1)]:
            res = O.run(g, params)
            assert res.K == r
            assert Fraction(res.N, res.D) == 1 - Fraction(1, r)
            for q in range(r):
                members = perm[q * s:(q + 1) * s]
                assert len(set(res.labels[members].tolist())) == 1


def p9_ring_of_cliques(O):
    """P9: a ring of r K_s joined by single edges; where the clique partition
    is optimal (brute force at (3,3); closed form elsewhere) the method
    recovers it and Q = 1 - 2/(s(s-1)+2) - 1/r."""
    g = SG.ring_of_cliques(3, 3)
    best, D = best_partition_N(g)
    assert Fraction(best, D) == Fraction(5, 12)
    for r, s in [(3, 3), (4, 5), (6, 5), (10, 6)]:
        g = SG.ring_of_cliques(r, s)
        res = O.run(g)
        closed = 1 - Fraction(2, s * (s - 1) + 2) - Fraction(1, r)
        assert res.K == r
        assert Fraction(res.N, res.D) == closed
        for q in range(r):
            assert len(set(res.labels[q * s:(q + 1) * s].tolist())) == 1


def p10_bruteforce_upper_bound(O):
    """P10: on graphs with <= 10 vertices the result never beats the best of
    all set partitions, and equals it on clear-structure cases."""
    import oracle as OR
    rng = np.random.default_rng(23)
    graphs = [SG.random_graph(rng, int(rng.integers(5, 9)), p=0.4, self_loops=0.2, wmax=5)
              for _ in range(6)]
    graphs.append(SG.random_graph(rng, 10, p=0.35, wmax=3))
    for g in graphs:
        best, D = best_partition_N(g)
        for params in [OR.Params(), OR.Params(vf=1, color=1, color_cutoff=1)]:
            res = O.run(g, params)
            if res.D != 1:
                assert res.D == D
            assert res.N <= best
    g = SG.cliques(2, 4)
    best, D = best_partition_N(g)
    assert O.run(g).N == best


def p11_coloring(O):
    """P11: the coloring is proper and every vertex has the smallest color not
    used by its higher-priority neighbours (this fixes it uniquely)."""
    mix64_published_check(O)
    rng = np.random.default_rng(29)
    seeds = [0x4C4F5556, 1, 12345]
    for gi, g in enumerate(rand_graphs(61, 8) + [SG.star(9), SG.cliques(3, 4)]):
        seed = seeds[gi % 3]
        st = O.state(g)
        nc = st.color(seed)
        col = st.get("color")
        assert nc == (int(col.max()) + 1 if g.n else 0)
        pri = [O.mix64(((seed << 32) ^ v) & ((1 << 64) - 1)) for v in range(g.n)]
        for v in range(g.n):
            nb = [int(u) for u in g.cols[g.offsets[v]:g.offsets[v + 1]] if u != v]
            assert all(col[u] != col[v] for u in nb)
            higher = {int(col[u]) for u in nb if pri[u] > pri[v]}
            mex = 0
            while mex in higher:
                mex += 1
            assert col[v] == mex


def p12_hand_cases(O):
    """P12: tiny cases worked by hand from Sec. 5.1's heuristics."""
    import oracle as OR
    # one edge: with the singlet rule only vertex 1 moves (to 0); without it the pair swaps
    g = SG.from_edges(2, [(0, 1)])
    res = O.run(g)
    assert res.phases[0].moves == [1, 0] and res.K == 1 and res.N == 0
    res = O.run(g, OR.Params(singlet_rule=0))
    assert res.phases[0].moves == [2, 2] and res.K == 2
    assert Fraction(res.N, res.D) == Fraction(-1, 2)
    # star: every leaf joins the hub's community; the hub's min-label target (leaf 1) is vetoed
    g = SG.star(6)
    st = O.state(g)
    assert st.decide(0, 1) == 0 and st.decide(0, 0) == 1
    assert all(st.decide(i, 1) == 0 for i in range(1, 7))
    res = O.run(g)
    assert res.phases[0].moves[0] == 6 and res.K == 1
    # clique with ties: every vertex but 0 picks label 0; 0 is vetoed from 1
    g = SG.cliques(1, 5)
    st = O.state(g)
    assert [st.decide(i, 1) for i in range(5)] == [0, 0, 0, 0, 0]
    assert [st.decide(i, 0) for i in range(5)] == [1, 0, 0, 0, 0]
    # VF: leaf follows its neighbour, an isolated pair merges into the smaller id
    g = SG.from_edges(7, [(0, 1), (1, 2), (2, 0), (3, 1), (4, 5), (6, 6)])
    st = O.state(g)
    st.vf()
    om = st.get("orig_map")
    assert om[3] == om[1] and om[4] == om[5] and len(set(om.tolist())) == 5
    assert st.info()["two_m"] == 2 * 5 + 1


def p13_rounding(O):
    """P13: the double is the correctly rounded N / D."""
    rng = np.random.default_rng(37)
    cases = [(1, 3), (2, 3), (-1, 3), (5, 12), ((1 << 53) + 1, 1 << 54), ((1 << 53) + 3, 1 << 54),
             (-((1 << 53) + 1), 1 << 54), (1, 1), (-1, 2), (0, 7)]
    for _ in range(300):
        D = int(rng.integers(1, 1 << 62)) * int(rng.integers(1, 1 << 62))
        N = int(rng.integers(-(1 << 62), 1 << 62)) * int(rng.integers(1, 1 << 62)) % D
        N = N if rng.random() < 0.5 else -N
        cases.append((N, D))
    for N, D in cases:
        assert O.ratio_to_double(N, D) == float(Fraction(N, D))


def p14_sbm_sanity(O):
    """P14 (plausibility): the 1,000-vertex planted partition is found,
    Q near its expected 0.746."""
    from paper_1410_1237_amd import graphs as G
    g = G.sbm_1000()
    res = O.run(g)
    assert res.K == 10
    assert abs(res.q - 0.746) < 0.01
    assert n_modmatrix(g, res.labels) == (res.N, res.D)


def validation_codes(O):
    g = SG.from_edges(3, [(0, 1), (1, 2)])
    assert O.validate(g) == 0
    bad = SG.from_edges(3, [(0, 1), (1, 2)])
    bad.cols = bad.cols.copy()
    bad.cols[0] = 2  # row 0 -> 2 has no mirror
    assert O.validate(bad) == 5
    bad2 = SG.from_edges(3, [(0, 1), (1, 2)], weights=[1, 2])
    bad2.weights = bad2.weights.copy()
    bad2.weights[0] = 0
    assert O.validate(bad2) == 4


def _trajectory(O, g, iters, singlet=1, color_seed=None):
    """N after each of `iters` iterations from the step calls, each checked
    against the modularity-matrix form of the partition it leaves."""
    st = O.state(g)
    if color_seed is not None:
        st.color(color_seed)
    out = []
    for _ in range(iters):
        _, N = st.iterate(singlet)
        assert N == n_modmatrix(g, st.get("comm"))[0]
        out.append(N)
    return out


def p15_loss_is_undone(O):
    """Sec. 5.1 (a phase continues only on a net gain) with Lemma 1 of
    Sec. 4.1 (simultaneous moves can lose): an iteration that lowers Q is not
    kept and ends the phase, also the first one of a phase.

    Case 1, a 4-cycle 0-1-2-3 with the chord 0-2 (k = 3,2,3,2; 2m = 10):
    singletons N0 = -(9+4+9+4) = -26.  Iteration 1 (by hand from Eq. 4 and
    the minimum-label rules): 0 prefers community 1 but the singlet rule
    keeps it, 1 and 3 join 0, 2 joins 1 -> {0,1,3},{2}: N = 10*4 - (49+9)
    = -18.  Iteration 2: 1 and 3 move to C(2), 2 moves to C(0) -> {0,2},{1,3}:
    N = 10*2 - (36+16) = -32, a loss.  So phase 1 ends at {0,1,3},{2} with
    N = -18 after 2 iterations; phase 2 merges the two (N = 0).

    Case 2, the 5-vertex graph 0-1, 0-4, 1-2, 1-3, 2-4, 3-4 (k = 2,3,2,2,3;
    2m = 12): N0 = -30.  Iteration 1 moves 1 and 4 to C(0), 2 and 3 to C(1)
    (0 is kept by the singlet rule) -> {0,1,4},{2,3}: N = 12*4 - (64+16) =
    -32 < -30.  The first iteration itself loses, so it is undone, the phase
    leaves every vertex alone, the graph does not shrink and the run stops at
    the singletons: K = 5, N = -30."""
    import oracle as OR
    g = SG.from_edges(4, [(0, 1), (0, 2), (0, 3), (1, 2), (2, 3)])
    assert _trajectory(O, g, 2) == [-18, -32]
    res = O.run(g, OR.Params(), phase_labels=True)
    p = res.phases[0]
    assert (p.iterations, p.moves, p.N_iter, p.N_end, p.undone) == (2, [3, 3], [-18, -32], -18, True)
    assert res.phase_labels[0].tolist() == [0, 0, 1, 0]
    assert res.phases[1].n == 2 and res.phases[1].N_end == 0
    assert (res.N, res.D, res.K) == (0, 100, 1)

    g = SG.from_edges(5, [(0, 1), (0, 4), (1, 2), (1, 3), (2, 4), (3, 4)])
    assert _trajectory(O, g, 1) == [-32]
    res = O.run(g)
    assert len(res.phases) == 1
    p = res.phases[0]
    assert (p.iterations, p.moves, p.N_end, p.undone) == (1, [4], -30, True)
    assert (res.N, res.K, res.N0) == (-30, 5, -30)
    assert res.labels.tolist() == [0, 1, 2, 3, 4]


def p16_phases_never_lose(O):
    """Consequence of the rule above: within a phase every kept iteration is
    at least the one before it, every phase ends at or above the N it started
    from (the previous phase's end, or the singletons' N0), and the run
    reports the last phase's N, checked on the modularity-matrix form."""
    import oracle as OR
    graphs = rand_graphs(71, 16) + [SG.ring_of_cliques(5, 4), SG.star(7)]
    for idx, g in enumerate(graphs):
        for params in [OR.Params(), OR.Params(singlet_rule=0),
                       OR.Params(vf=1, color=1, color_cutoff=1, theta_color=(1, 4))]:
            res = O.run(g, params, phase_labels=True)
            prev = res.N0
            for ph, lab in zip(res.phases, res.phase_labels):
                kept = ph.N_iter[:-1] if ph.undone else ph.N_iter
                seq = [prev] + kept
                assert all(b >= a for a, b in zip(seq, seq[1:]))
                if ph.undone:
                    assert ph.N_iter[-1] < seq[-1]
                assert ph.N_end == seq[-1] >= prev
                assert n_modmatrix(g, lab)[0] == ph.N_end
                prev = ph.N_end
            assert res.N == prev


def p17_iteration_threshold(O):
    """Alg. 1's threshold test, in exact rationals.  On the 5-vertex graph
    0-1, 0-4, 1-2, 1-3, 2-3, 2-4 (2m = 12, D = 144) the iterations give
    N = -14, 0, 16, 16 (moves 3, 3, 1, 0).
      * relative test (gain against theta * |N_{t-1}|), theta = 1/2:
        t = 2 gains 14 >= 7, t = 3 gains 16 >= 0, t = 4 moves nothing ->
        4 iterations;
      * absolute test (gain against theta * D), theta = 1/2: t = 2 gains
        14 < 72 -> stops after 2 iterations;
      * the test is strict: theta = 14/14 puts t = 2 exactly on the
        threshold and the phase goes on (4 iterations); theta = 15/14 stops
        it at t = 2;
      * t = 1 is never tested (Alg. 1 starts from Q_P = -infinity): even
        theta = 10^6 keeps iteration 1 and stops at t = 2."""
    import oracle as OR
    g = SG.from_edges(5, [(0, 1), (0, 4), (1, 2), (1, 3), (2, 3), (2, 4)])
    assert _trajectory(O, g, 4) == [-14, 0, 16, 16]
    runs = {"rel": OR.Params(theta_final=(1, 2)),
            "abs": OR.Params(theta_final=(1, 2), threshold_mode=1),
            "at": OR.Params(theta_final=(14, 14)),
            "above": OR.Params(theta_final=(15, 14)),
            "huge": OR.Params(theta_final=(10 ** 6, 1))}
    first = {k: O.run(g, P).phases[0] for k, P in runs.items()}
    assert (first["rel"].iterations, first["rel"].N_end) == (4, 16)
    assert (first["abs"].iterations, first["abs"].N_end) == (2, 0)
    assert (first["at"].iterations, first["at"].N_end) == (4, 16)
    assert (first["above"].iterations, first["above"].N_end) == (2, 0)
    assert (first["huge"].iterations, first["huge"].moves) == (2, [3, 3])


def p18_coloring_schedule(O):
    """Sec. 6.1's schedule.  The 5-vertex graph 0-2, 0-3, 1-2, 1-3, 2-3,
    2-4, 3-4 (k = 2,2,4,4,2; 2m = 14; N0 = -44) colored with the default
    seed gives N = -20, -8, 0, 0 per iteration (gains 24, 12, 8, 0).
      * theta_color = 9/10 governs a colored phase: t = 2 gains 12 < 18
        and stops it (theta_final = 1e-6 would run to t = 4);
      * the phase gain is then -8 - (-44) = 36 < 0.9 * 44, so coloring
        stops: phase 2 runs uncolored although its graph (2 vertices) is
        above the cutoff of 1;
      * a phase is colored when its graph has at least `color_cutoff`
        vertices: cutoff 5 colors the 5-vertex phase, cutoff 6 does not;
      * with color_first_phase_only (Table 4's variant) phase 2 is
        uncolored even though phase 1 gained 44 >= 0.01 * 44."""
    import oracle as OR
    g = SG.from_edges(5, [(0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (2, 4), (3, 4)])
    assert _trajectory(O, g, 4, color_seed=OR.DEFAULT_SEED) == [-20, -8, 0, 0]
    res = O.run(g, OR.Params(color=1, color_cutoff=1, theta_color=(9, 10)))
    assert [(p.colored, p.iterations, p.N_end) for p in res.phases[:2]] == [(True, 2, -8), (False, 2, 0)]
    res = O.run(g, OR.Params(color=1, color_cutoff=5, theta_color=(9, 10)))
    assert res.phases[0].colored and res.phases[0].iterations == 2
    res = O.run(g, OR.Params(color=1, color_cutoff=6, theta_color=(9, 10)))
    assert not res.phases[0].colored
    res = O.run(g, OR.Params(color=1, color_cutoff=1))
    assert [p.colored for p in res.phases[:2]] == [True, True] and res.phases[0].iterations == 4
    res = O.run(g, OR.Params(color=1, color_cutoff=1, color_first_phase_only=1))
    assert [p.colored for p in res.phases] == [True, False]


def p19_no_shrink_stops(O):
    """A phase that leaves every community a single vertex cannot shrink the
    graph, and gains nothing (its partition is the singletons again).  With
    the thresholds at 0 only that rule ends the run:
      * uncolored: the 5-vertex graph 0-1, 0-4, 1-2, 1-3, 2-4, 3-4 has its
        first iteration undone (p15), so phase 1 does not shrink: 1 phase;
      * colored (cutoff 1, theta_color = 0): the phases shrink 5 -> 2 -> 1;
        the 1-vertex phase does not shrink, which ends coloring, and the
        uncolored phase after it does not shrink either: 4 phases, the last
        uncolored."""
    import oracle as OR
    g = SG.from_edges(5, [(0, 1), (0, 4), (1, 2), (1, 3), (2, 4), (3, 4)])
    res = O.run(g, OR.Params(theta_final=(0, 1)))
    assert len(res.phases) == 1 and res.K == 5
    res = O.run(g, OR.Params(color=1, color_cutoff=1, theta_color=(0, 1), theta_final=(0, 1)))
    assert [(p.n, p.colored) for p in res.phases] == [(5, True), (2, True), (1, True), (1, False)]


def p20_vf_isolated_pair(O):
    """Sec. 5.3 with the isolated-pair reading: both ends of an isolated edge
    (2, 7) follow the smaller id, so the rebuilt graph keeps vertex 2's rank:
    representatives 0,1,2,3,4,5,6,8,9 are renumbered 0..8, hence 2 and 7 map
    to 2 and 8 -> 7, 9 -> 8.  Triangles 0-1-3, 4-5-6, 0-8-9 keep every other
    vertex."""
    g = SG.from_edges(10, [(0, 1), (0, 3), (1, 3), (4, 5), (4, 6), (5, 6), (0, 8), (0, 9), (8, 9), (2, 7)])
    st = O.state(g)
    st.vf()
    assert st.get("orig_map").tolist() == [0, 1, 2, 3, 4, 5, 6, 2, 7, 8]
    off, cols, w = st.get("offsets"), st.get("cols"), st.get("weights")
    row2 = (cols[off[2]:off[3]].tolist(), w[off[2]:off[3]].tolist())
    assert row2 == ([2], [2])   # the pair's edge, both entries, as a self-loop


def _chain_qualifies(n, off, cols, w):
    """Vertices of a CSR that the chain rule would still merge: one
    neighbour j != i (a self-loop allowed) and 2m * w_ij > k_i * k_j."""
    k = np.array([int(w[off[i]:off[i + 1]].sum()) for i in range(n)], dtype=object)
    two_m = int(sum(k))
    out = []
    for i in range(n):
        nb = [(int(c), int(x)) for c, x in zip(cols[off[i]:off[i + 1]], w[off[i]:off[i + 1]]) if c != i]
        if len(nb) == 1 and two_m * nb[0][1] > k[i] * k[nb[0][0]]:
            out.append(i)
    return out


def p21_chain_vertex_following(O):
    """The chain-compressing extension of Sec. 5.3: single-neighbour vertices
    merge into their neighbour round after round while the bound of Lemma 3's
    proof stays positive, 2m * w_ij > k_i * k_j.

      * path 0-1-2-3 ending in the triangle 3-4-5 (unit weights, 2m = 12):
        round 1 merges the leaf 0 into 1 (12 > 1*2); {0,1} now has a
        self-loop of 2 and the single neighbour 2, and 12 > 3*2 merges it into
        2; {0,1,2} (self-loop 4, k = 5) with neighbour 3 (k = 3) gives
        12 > 15, false: two rounds, map 0,0,0,1,2,3, self-loop 4;
      * a vertex with a self-loop of 10 and one edge into a triangle
        (2m = 18): 18 * 1 > 11 * 3 is false, nothing merges; with a self-loop
        of 2 (2m = 10): 10 > 3 * 3 merges it;
      * an isolated pair whose ends carry self-loops of 1 (2m = 10 with a
        triangle beside it): both qualify (10 > 2*2) and go to the smaller
        id; the merged self-loop is 1 + 1 + 2 * 1 = 4.
    On random graphs the rounds keep 2m and Q (the partition of the original
    graph by the composed map has the rebuilt graph's singleton Q), and no
    vertex of the result qualifies any more."""
    g = SG.from_edges(6, [(0, 1), (1, 2), (2, 3), (3, 4), (3, 5), (4, 5)])
    st = O.state(g)
    assert st.vf_chain() == 2
    assert st.get("orig_map").tolist() == [0, 0, 0, 1, 2, 3]
    off, cols, w = st.get("offsets"), st.get("cols"), st.get("weights")
    assert (cols[off[0]:off[1]].tolist(), w[off[0]:off[1]].tolist()) == ([0, 1], [4, 1])
    for sw, rounds, om in [(10, 0, [0, 1, 2, 3]), (2, 1, [0, 0, 1, 2])]:
        g = SG.from_edges(4, [(0, 0), (0, 1), (1, 2), (1, 3), (2, 3)], [sw, 1, 1, 1, 1])
        st = O.state(g)
        assert st.vf_chain() == rounds and st.get("orig_map").tolist() == om
    g = SG.from_edges(5, [(0, 0), (0, 1), (1, 1), (2, 3), (2, 4), (3, 4)])
    st = O.state(g)
    assert st.vf_chain() == 1 and st.get("orig_map").tolist() == [0, 0, 1, 2, 3]
    assert st.get("weights")[0] == 4
    # the bound is strict: self-loop 6 and an edge of weight 2 into a triangle
    # give 2m = 16, k_0 = 8, k_1 = 4 and 16 * 2 = 8 * 4: no merge
    g = SG.from_edges(4, [(0, 0), (0, 1), (1, 2), (1, 3), (2, 3)], [6, 2, 1, 1, 1])
    st = O.state(g)
    assert st.vf_chain() == 0 and st.get("orig_map").tolist() == [0, 1, 2, 3]
    # an isolated pair with non-adjacent ids (2, 7) follows the smaller id here too
    g = SG.from_edges(10, [(0, 1), (0, 3), (1, 3), (4, 5), (4, 6), (5, 6), (0, 8), (0, 9), (8, 9), (2, 7)])
    st = O.state(g)
    assert st.vf_chain() == 1 and st.get("orig_map").tolist() == [0, 1, 2, 3, 4, 5, 6, 2, 7, 8]
    # single-degree VF on the path case takes the leaf only
    st = O.state(SG.from_edges(6, [(0, 1), (1, 2), (2, 3), (3, 4), (3, 5), (4, 5)]))
    st.vf()
    assert st.get("orig_map").tolist() == [0, 0, 1, 2, 3, 4]
    rng = np.random.default_rng(43)
    for t in range(24):
        n = int(rng.integers(4, 16))
        g = SG.random_graph(rng, n, p=float(rng.uniform(0.08, 0.3)), self_loops=0.3 if t % 2 else 0.0,
                            wmax=1 if t % 3 == 0 else 6)
        if g.nnz == 0:
            continue
        st = O.state(g)
        two_m = st.info()["two_m"]
        st.vf_chain()
        info = st.info()
        off, cols, w = st.get("offsets"), st.get("cols"), st.get("weights")
        _check_csr(info["n"], off, cols, w)
        assert info["two_m"] == two_m
        A2 = dense_w64(info["n"], off, cols, w)
        assert n_modmatrix(g, st.get("orig_map")) == n_modmatrix_A(A2, np.arange(info["n"]))
        assert _chain_qualifies(info["n"], off, cols, w) == []


def p22_balanced_coloring(O):
    """Balanced colouring (class-size equalisation of the greedy colouring).
    A triangle 0-1-2 beside 7 isolated vertices 3..9: the greedy colouring
    has chi = 3 (the triangle) and puts every isolated vertex in class 0, so
    |K_0| = 8, |K_1| = |K_2| = 1 and gamma = ceil(10 / 3) = 4.  The triangle's
    vertex in K_0 sees colours 1 and 2 and cannot move; the isolated ones can
    go anywhere.  Round 1: all propose colour 1, which takes 3 (4 - 1) in
    descending priority, within the room of 8 - 4 = 4: they move.  Round 2: the
    other 4 propose colour 2, which could take 3, but only 1 more may leave
    K_0: the highest-priority one moves.  Sizes 4, 4, 2.
    On random graphs: still proper, no new colour, no class pushed past gamma,
    and a vertex left in a class above gamma has no admissible colour."""
    g = SG.from_edges(10, [(0, 1), (0, 2), (1, 2)])
    st = O.state(g)
    seed = 0x4C4F5556
    assert st.color(seed) == 3
    before = st.get("color")
    assert (before[3:] == 0).all()
    assert st.balance(seed) == 4
    after = st.get("color")
    pri = {v: O.mix64(((seed << 32) ^ v) & ((1 << 64) - 1)) for v in range(3, 10)}
    iso = sorted(range(3, 10), key=lambda v: -pri[v])
    assert [int(after[v]) for v in iso] == [1, 1, 1, 2, 0, 0, 0]
    assert np.array_equal(after[:3], before[:3])
    assert np.bincount(after, minlength=3).tolist() == [4, 4, 2]
    rng = np.random.default_rng(53)
    for t in range(20):
        n = int(rng.integers(6, 40))
        g = SG.random_graph(rng, n, p=float(rng.uniform(0.03, 0.4)), self_loops=0.2 if t % 2 else 0.0)
        st = O.state(g)
        chi = st.color(seed)
        size0 = np.bincount(st.get("color"), minlength=chi)
        st.balance(seed)
        col = st.get("color")
        assert col.max() < chi
        gamma = -(-n // chi)
        size1 = np.bincount(col, minlength=chi)
        assert all(size1[c] <= max(gamma, size0[c]) for c in range(chi))
        for v in range(n):
            nb = [int(u) for u in g.cols[g.offsets[v]:g.offsets[v + 1]] if u != v]
            assert all(col[u] != col[v] for u in nb)
            if size1[col[v]] > gamma:
                used = {int(col[u]) for u in nb}
                assert not [d for d in range(chi) if d != col[v] and size1[d] < gamma and d not in used]


ALL = [p1_singleton_closed_form, p2_totals_invariant, p3_single_move_is_eq4, p4_eq6_two_moves,
       p5_lemma3, p6_coarsen_invariance, p7_phase_q_from_scratch, p8_disjoint_cliques,
       p9_ring_of_cliques, p10_bruteforce_upper_bound, p11_coloring, p12_hand_cases,
       p13_rounding, p14_sbm_sanity, validation_codes, p15_loss_is_undone, p16_phases_never_lose,
       p17_iteration_threshold, p18_coloring_schedule, p19_no_shrink_stops, p20_vf_isolated_pair,
       p21_chain_vertex_following, p22_balanced_coloring]
