"""GPU path vs the oracle, bit for bit, through the C ABI.

Step level: degrees, vertex following, coloring, every synchronous sweep
(communities, community degrees and sizes, moves, modularity numerator)
and every rebuild (CSR byte-equal, composed map).  Run level: labels, K,
exact (N, D), the double, per-phase sizes, iteration counts, per-iteration
moves and N.  Inputs: seeded small random graphs with self-loops and
weights, a star large enough for the hub bin, SBM, R-MAT, Chung-Lu, and the
degenerate cases.
"""
import numpy as np
import pytest

import oracle
import small_graphs as SG
from paper_1410_1237_amd import graphs as GG

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available()
    from paper_1410_1237_amd import louvain
    louvain.lib()
    return louvain


@pytest.fixture(scope="module")
def O():
    return oracle.default()


def hub_graph(seed=3, hub_deg=5000, extra=20000, n=8000):
    """A random graph with one vertex of degree hub_deg (hub bins) and a few of degree 300-900."""
    rng = np.random.default_rng(seed)
    edges = set()
    for v in rng.choice(np.arange(1, n), size=hub_deg, replace=False):
        edges.add((0, int(v)))
    for h in (1, 2, 3):
        for v in rng.choice(np.arange(4, n), size=300 * h, replace=False):
            edges.add((min(h, int(v)), max(h, int(v))))
    while len(edges) < hub_deg + extra:
        u, v = (int(x) for x in rng.integers(0, n, 2))
        if u != v:
            edges.add((min(u, v), max(u, v)))
    edges = sorted(edges)
    w = rng.integers(1, 20, size=len(edges))
    return SG.from_edges(n, edges, w, name="hub_graph")


def small_cases():
    rng = np.random.default_rng(101)
    gs = []
    for t in range(6):
        n = int(rng.integers(5, 60))
        gs.append(SG.random_graph(rng, n, p=float(rng.uniform(0.05, 0.5)), self_loops=0.3 if t % 2 else 0.0,
                                  wmax=1 if t % 3 == 0 else 9))
    gs.append(SG.ring_of_cliques(6, 5))
    gs.append(SG.star(40))
    return gs


def medium_cases():
    return [GG.sbm_1000(), GG.rmat(12, 8, seed=5), GG.rmat(13, 16, wmax=100, seed=6), hub_graph(),
            GG.chung_lu(20000, 2.1, 2000.0, 3.0e5, 150000, wmax=100, seed=4), GG.batch_sbm(7),
            hub_graph(seed=11, hub_deg=40000, extra=60000, n=50000)]


def expand_w(g):
    return np.ones(g.nnz, np.int64) if g.weights is None else g.weights.astype(np.int64)


def compare_state(gs, st, tag):
    s = gs.state()
    assert np.array_equal(s["comm"], st.get("comm")), tag + ": communities"
    assert np.array_equal(s["a"], st.get("a")), tag + ": community degrees"
    assert np.array_equal(s["size"], st.get("size")), tag + ": community sizes"
    assert np.array_equal(s["k"], st.get("k")), tag + ": degrees"


def compare_graph(gs, st, tag):
    off, col, w = gs.graph()
    assert np.array_equal(off, st.get("offsets")), tag + ": offsets"
    assert np.array_equal(col, st.get("cols")), tag + ": cols"
    assert np.array_equal(w, st.get("weights")), tag + ": weights"
    assert np.array_equal(gs.orig_map(), st.get("orig_map")), tag + ": map"


@pytest.mark.parametrize("case", range(8))
def test_steps_small(L, O, case):
    g = small_cases()[case]
    _steps(L, O, g, colored=(case % 2 == 1), vf=(case % 3 == 0))


@pytest.mark.parametrize("colored", [False, True])
@pytest.mark.parametrize("case", range(7))
def test_steps_medium(L, O, case, colored):
    g = medium_cases()[case]
    _steps(L, O, g, colored=colored, vf=(case % 3 != 1), phases=2, iters=4)


def _steps(L, O, g, colored, vf, phases=3, iters=6):
    print(f"[steps] {g.name} n={g.n} nnz={g.nnz} colored={colored} vf={vf}", flush=True)
    gs = L.Graph.from_csr(g)
    st = O.state(g)
    info = gs.info()
    assert info["two_m"] == st.info()["two_m"]
    compare_state(gs, st, "init")
    if vf:
        n1 = gs.vf()
        st.vf()
        assert n1 == st.info()["n"]
        compare_graph(gs, st, "vf")
        compare_state(gs, st, "vf")
    p = L.params(color=1 if colored else 0)
    for ph in range(phases):
        if colored:
            c1 = gs.color()
            c2 = st.color()
            assert c1 == c2
            assert np.array_equal(gs.colors(), st.get("color")), "colors"
        else:
            st.uncolor()
        for t in range(iters):
            r = gs.sweep(p)
            moves, N = st.iterate(1)
            tag = f"phase {ph} iteration {t}"
            assert r["moves"] == moves, tag + ": moves"
            assert r["N"] == N, tag + ": modularity numerator"
            compare_state(gs, st, tag)
            if moves == 0:
                break
        n1 = gs.coarsen()
        n2 = st.coarsen()
        assert n1 == n2
        compare_graph(gs, st, f"coarsen {ph}")
        compare_state(gs, st, f"coarsen {ph}")
    gs.close()


def compare_run(res, ref, tag=""):
    assert res.K == ref.K, tag + ": K"
    assert (res.N, res.D) == (ref.N, ref.D), tag + ": exact modularity"
    assert res.q == ref.q, tag + ": double"
    assert res.N0 == ref.N0 and res.n_vf == ref.n_vf, tag + ": first phase"
    assert len(res.phases) == len(ref.phases), tag + ": phases"
    for a, b in zip(res.phases, ref.phases):
        assert (a.n, a.nnz, a.colored, a.num_colors, a.iterations, a.hit_max_iter, a.undone) == \
               (b.n, b.nnz, b.colored, b.ncolors, b.iterations, b.hit_max_iter, b.undone), tag + ": phase shape"
        assert a.moves == b.moves, tag + ": moves"
        assert a.N_iter == b.N_iter, tag + ": per-iteration modularity"
        assert a.N_end == b.N_end, tag + ": phase modularity"
    assert np.array_equal(res.labels, ref.labels), tag + ": labels"


PARAM_SETS = [
    dict(),
    dict(singlet_rule=0),
    dict(vf=1, color=1, color_cutoff=1),
    dict(vf=1, color=1, color_cutoff=1, color_first_phase_only=1),
    dict(vf=1, color=1, color_cutoff=50, theta_color=(1, 10000)),
    dict(threshold_mode=1, theta_final=(1, 1000)),
    dict(max_iter=2, max_phases=2),
]


def oracle_params(d):
    return oracle.Params(**d)


@pytest.mark.parametrize("pi", range(len(PARAM_SETS)))
def test_run_small(L, O, pi):
    for g in small_cases():
        res = L.Graph.from_csr(g).run(L.params(**PARAM_SETS[pi]))
        ref = O.run(g, oracle_params(PARAM_SETS[pi]))
        compare_run(res, ref, f"{g.name} {PARAM_SETS[pi]}")


@pytest.mark.parametrize("case", range(7))
def test_run_medium(L, O, case):
    g = medium_cases()[case]
    for d in (dict(), dict(vf=1, color=1, color_cutoff=1000)):
        print(f"[run] {g.name} {d}", flush=True)
        with L.Graph.from_csr(g) as gs:
            res = gs.run(L.params(**d))
        compare_run(res, O.run(g, oracle_params(d)), f"{g.name} {d}")


STOP_RULE_CASES = [
    # (vertices, edges, params): the hand-worked cases of the oracle's
    # stop-rule and schedule pins (a loss undone at t = 2 and at t = 1,
    # relative/absolute/strict thresholds, theta_color, cutoff, no-shrink)
    (4, [(0, 1), (0, 2), (0, 3), (1, 2), (2, 3)], dict()),
    (5, [(0, 1), (0, 4), (1, 2), (1, 3), (2, 4), (3, 4)], dict()),
    (5, [(0, 1), (0, 4), (1, 2), (1, 3), (2, 4), (3, 4)], dict(theta_final=(0, 1))),
    (5, [(0, 1), (0, 4), (1, 2), (1, 3), (2, 4), (3, 4)],
     dict(color=1, color_cutoff=1, theta_color=(0, 1), theta_final=(0, 1))),
    (5, [(0, 1), (0, 4), (1, 2), (1, 3), (2, 3), (2, 4)], dict(theta_final=(1, 2))),
    (5, [(0, 1), (0, 4), (1, 2), (1, 3), (2, 3), (2, 4)], dict(theta_final=(1, 2), threshold_mode=1)),
    (5, [(0, 1), (0, 4), (1, 2), (1, 3), (2, 3), (2, 4)], dict(theta_final=(14, 14))),
    (5, [(0, 1), (0, 4), (1, 2), (1, 3), (2, 3), (2, 4)], dict(theta_final=(15, 14))),
    (5, [(0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (2, 4), (3, 4)], dict(color=1, color_cutoff=1, theta_color=(9, 10))),
    (5, [(0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (2, 4), (3, 4)], dict(color=1, color_cutoff=5, theta_color=(9, 10))),
    (5, [(0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (2, 4), (3, 4)], dict(color=1, color_cutoff=6, theta_color=(9, 10))),
    (5, [(0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (2, 4), (3, 4)],
     dict(color=1, color_cutoff=1, color_first_phase_only=1)),
    (10, [(0, 1), (0, 3), (1, 3), (4, 5), (4, 6), (5, 6), (0, 8), (0, 9), (8, 9), (2, 7)], dict(vf=1)),
]


@pytest.mark.parametrize("case", range(len(STOP_RULE_CASES)))
def test_run_stop_rule_cases(L, O, case):
    n, edges, d = STOP_RULE_CASES[case]
    g = SG.from_edges(n, edges)
    res = L.Graph.from_csr(g).run(L.params(**d))
    compare_run(res, O.run(g, oracle_params(d)), f"stop-rule case {case} {d}")


def chain_graph(seed=9, n=3000):
    """A sparse random graph with hanging paths of several lengths and some
    self-loops, so that chain rounds merge, stop on the bound and repeat."""
    rng = np.random.default_rng(seed)
    edges, ws = set(), {}
    core = n // 3
    while len(edges) < 3 * core:
        u, v = (int(x) for x in rng.integers(0, core, 2))
        if u != v:
            edges.add((min(u, v), max(u, v)))
    nxt = core
    while nxt < n:
        length = int(rng.integers(1, 12))
        prev = int(rng.integers(0, core))
        for _ in range(length):
            if nxt >= n:
                break
            edges.add((min(prev, nxt), max(prev, nxt)))
            prev = nxt
            nxt += 1
    for v in rng.choice(n, size=n // 20, replace=False):
        edges.add((int(v), int(v)))
    edges = sorted(edges)
    w = rng.integers(1, 9, size=len(edges))
    return SG.from_edges(n, edges, w, name="chain_graph")


@pytest.mark.parametrize("case", range(4))
def test_vf_chain_steps(L, O, case):
    """Chain-compressing vertex following through the step call: the
    rebuilt graph (CSR byte-equal), the composed map and the round count
    equal the oracle's, then one phase of sweeps."""
    g = [chain_graph(), chain_graph(seed=10, n=20000), SG.ring_of_cliques(6, 5), GG.rmat(12, 4, seed=3)][case]
    gs = L.Graph.from_csr(g)
    st = O.state(g)
    n1, r1 = gs.vf_chain()
    r2 = st.vf_chain()
    assert (n1, r1) == (st.info()["n"], r2)
    compare_graph(gs, st, "vf chain")
    compare_state(gs, st, "vf chain")
    p = L.params()
    for t in range(4):
        r = gs.sweep(p)
        moves, N = st.iterate(1)
        assert (r["moves"], r["N"]) == (moves, N)
        compare_state(gs, st, f"iteration {t}")
        if moves == 0:
            break
    gs.close()


@pytest.mark.parametrize("d", [dict(vf=2), dict(vf=2, color=1, color_cutoff=1000)])
def test_run_vf_chain(L, O, d):
    for g in small_cases() + [chain_graph(), chain_graph(seed=10, n=20000), GG.rmat(13, 4, wmax=20, seed=4)]:
        res = L.Graph.from_csr(g).run(L.params(**d))
        ref = O.run(g, oracle_params(d))
        compare_run(res, ref, f"{g.name} {d}")
        assert res.vf_rounds == ref.vf_rounds


@pytest.mark.parametrize("case", range(5))
def test_balanced_coloring_steps(L, O, case):
    """Balanced colouring through the step call: the colours after balancing
    and the moved count equal the oracle's, then the coloured sweeps."""
    rng = np.random.default_rng(200 + case)
    g = [SG.from_edges(10, [(0, 1), (0, 2), (1, 2)]), SG.random_graph(rng, 300, p=0.02, self_loops=0.1),
         GG.rmat(12, 8, seed=5), hub_graph(), GG.rmat(14, 16, wmax=10, seed=7)][case]
    gs = L.Graph.from_csr(g)
    st = O.state(g)
    assert gs.color() == st.color()
    assert gs.balance() == st.balance()
    assert np.array_equal(gs.colors(), st.get("color")), "balanced colours"
    p = L.params(color=1)
    for t in range(3):
        r = gs.sweep(p)
        moves, N = st.iterate(1)
        assert (r["moves"], r["N"]) == (moves, N)
        compare_state(gs, st, f"iteration {t}")
        if moves == 0:
            break
    gs.close()


def test_run_balanced_coloring(L, O):
    d = dict(vf=1, color=1, color_cutoff=50, color_balance=1)
    for g in small_cases() + [GG.rmat(12, 8, seed=5), hub_graph(), GG.sbm_1000()]:
        res = L.Graph.from_csr(g).run(L.params(**d))
        compare_run(res, O.run(g, oracle_params(d)), f"{g.name} {d}")


def test_clique_beyond_4096_colours(L, O):
    """A clique of 4,200 vertices needs 4,200 colours: the last vertices to
    be coloured see all of the first 4,096 colours taken by higher-priority
    neighbours, which sends their long rows past the 4,096-bit bitmap to the
    64-colour-window continuation.  Colours equal the oracle's greedy ones."""
    n = 4200
    full = np.tile(np.arange(n, dtype=np.int32), (n, 1))
    cols = full[~np.eye(n, dtype=bool)]                  # row-major, ascending within each row
    off = np.arange(n + 1, dtype=np.int64) * (n - 1)
    g = SG.CSR(n=n, offsets=off, cols=np.ascontiguousarray(cols), weights=None, name="clique_4200")
    gs = L.Graph.from_csr(g, validate=False)
    st = O.state(g)
    assert gs.color() == st.color() == n
    assert np.array_equal(gs.colors(), st.get("color"))
    gs.close()


def boundary_graph(seed):
    """Rows at the colouring's length limits: vertices of degree exactly 256
    and 257 (light/long), 1024/1025 and 2048/2049 (one/two/three chunks),
    a clique of 150 light rows (colours past 64 in a wavefront's bitmap), a
    clique of 300 long rows (long rows adjacent to long rows in both
    priority directions) with 100 light vertices tied to 200 of its members
    each (light rows seeing ~200 colours, long rows with light higher- and
    lower-priority neighbours), and random edges."""
    rng = np.random.default_rng(seed)
    n = 6000
    edges = set()

    def add(u, v):
        if u != v:
            edges.add((min(u, v), max(u, v)))

    for h, d in enumerate((256, 257, 1024, 1025, 2048, 2049, 3000)):
        for v in rng.choice(np.arange(10, n), size=d, replace=False):
            add(h, int(v))
    for a in range(10, 160):
        for b in range(a + 1, 160):
            add(a, b)
    for a in range(200, 500):
        for b in range(a + 1, 500):
            add(a, b)
    for v in range(600, 700):
        for u in rng.choice(np.arange(200, 500), size=200, replace=False):
            add(v, int(u))
    while len(edges) < 140000:
        u, v = (int(x) for x in rng.integers(10, n, 2))
        add(u, v)
    return SG.from_edges(n, sorted(edges), None, name=f"boundary_graph_{seed}")


@pytest.mark.parametrize("seed", [1, 2])
def test_colouring_row_length_boundaries(L, O, seed):
    g = boundary_graph(seed)
    deg = np.diff(g.offsets)
    assert list(deg[:7]) == [256, 257, 1024, 1025, 2048, 2049, 3000]
    gs = L.Graph.from_csr(g)
    st = O.state(g)
    for colouring in range(2):
        # the second colouring (another seed) reuses the bitmaps and lists
        seed_c = L.DEFAULT_SEED + colouring
        assert gs.color(seed_c) == st.color(seed_c)
        assert np.array_equal(gs.colors(), st.get("color")), f"colours, seed {seed_c}"
    gs.close()
    d = dict(vf=0, color=1, color_cutoff=1)
    res = L.Graph.from_csr(g).run(L.params(**d))
    compare_run(res, O.run(g, oracle_params(d)), g.name)


def test_run_sbm_1000(L, O):
    g = GG.sbm_1000()
    res = L.Graph.from_csr(g).run(L.params())
    ref = O.run(g)
    compare_run(res, ref, "sbm_1000")
    assert res.K == 10


def test_repeat_and_device_labels(L, O):
    import torch
    g = GG.rmat(12, 16, seed=9)
    gs = L.Graph.from_csr(g)
    a = gs.run(L.params(vf=1, color=1, color_cutoff=100))
    b = gs.run(L.params(vf=1, color=1, color_cutoff=100))
    lab = torch.zeros(g.n, dtype=torch.int32, device="cuda")
    c = gs.run(L.params(vf=1, color=1, color_cutoff=100), labels=lab)
    torch.cuda.synchronize()
    assert np.array_equal(a.labels, b.labels) and np.array_equal(a.labels, lab.cpu().numpy())
    assert (a.N, b.N, c.N) == (a.N, a.N, a.N)
    gs.close()


def test_device_pointer_ingest(L, O):
    import torch
    g = GG.rmat(11, 8, wmax=50, seed=2)
    off = torch.from_numpy(g.offsets).cuda()
    col = torch.from_numpy(g.cols).cuda()
    w = torch.from_numpy(g.weights).cuda()
    gs = L.Graph.from_tensors(off, col, w, validate=True)
    compare_run(gs.run(L.params()), O.run(g), "device ingest")
    gs.close()


def test_degenerate(L, O):
    cases = [SG.from_edges(0, []), SG.from_edges(1, []), SG.from_edges(5, []),
             SG.from_edges(3, [(0, 0), (2, 2)], weights=[3, 4]), SG.from_edges(2, [(0, 1)]),
             SG.from_edges(4, [(0, 1), (2, 3)]), SG.from_edges(6, [(0, 1), (1, 2), (4, 4)])]
    for g in cases:
        for d in (dict(), dict(vf=1, color=1, color_cutoff=1), dict(singlet_rule=0)):
            res = L.Graph.from_csr(g).run(L.params(**d))
            compare_run(res, O.run(g, oracle_params(d)), f"degenerate n={g.n} {d}")


def test_bad_csr_rejected(L):
    g = SG.from_edges(4, [(0, 1), (1, 2), (2, 3)], weights=[1, 2, 3])
    bad = [("asym", lambda c: c.weights.__setitem__(0, 5)), ("range", lambda c: c.cols.__setitem__(0, 9)),
           ("order", lambda c: c.cols.__setitem__(slice(1, 3), c.cols[1:3][::-1].copy())),
           ("weight", lambda c: (c.weights.__setitem__(0, 0), c.weights.__setitem__(1, 0)))]
    for name, mutate in bad:
        c = SG.from_edges(4, [(0, 1), (1, 2), (2, 3)], weights=[1, 2, 3])
        c.cols = c.cols.copy()
        c.weights = c.weights.copy()
        mutate(c)
        with pytest.raises(L.LouvainError) as e:
            L.Graph.from_csr(c)
        assert e.value.status == L.E_BAD_CSR, name
    # without full validation the column range is still checked (by the degree pass)
    for bad_col, at in ((7, 0), (-1, 0), (4, 5)):
        c = SG.from_edges(4, [(0, 1), (1, 2), (2, 3)])
        c.cols = c.cols.copy()
        c.cols[at] = bad_col
        with pytest.raises(L.LouvainError) as e:
            L.Graph.from_csr(c, validate=False)
        assert e.value.status == L.E_BAD_CSR, (bad_col, at)
    L.Graph.from_csr(g).close()


def test_profiling_records(L):
    g = GG.rmat(12, 16, seed=4)
    gs = L.Graph.from_csr(g)
    gs.profile(True)
    res = gs.run(L.params())
    recs = {r["name"]: r for r in gs.profile_records()}
    swept = sum(r["entries"] for n, r in recs.items() if n.startswith("sweep"))
    assert swept == res.sweep_entries + res.lookahead_entries
    assert all(r["ms"] >= 0 for r in recs.values())
    gs.close()


def overflow_hub_graph(seed=17, n=100_000, extra=50_000):
    """Hubs whose neighbours' communities all fall in one hash bucket, so a
    bucket holds more distinct communities than one aggregation round may
    (degree 4,000 in bucket 0 of 2, degree 9,000 in bucket 0 of 8): their
    buckets are summed in several rounds."""
    rng = np.random.default_rng(seed)
    ids = np.arange(2, n, dtype=np.uint64)
    fib = (ids * np.uint64(0x9E3779B1)) & np.uint64(0xFFFFFFFF)
    edges = set()
    for hub, deg, bits in ((0, 4000, 1), (1, 9000, 3)):
        pool = ids[(fib >> np.uint64(32 - bits)) == 0]
        for v in rng.choice(pool, size=deg, replace=False):
            edges.add((hub, int(v)))
    while len(edges) < 13000 + extra:
        u, v = (int(x) for x in rng.integers(2, n, 2))
        if u != v:
            edges.add((min(u, v), max(u, v)))
    edges = sorted(edges)
    w = rng.integers(1, 30, size=len(edges))
    return SG.from_edges(n, edges, w, name="overflow_hub_graph")


@pytest.mark.parametrize("pi", [0, 2])
def test_hub_bucket_overflow(L, O, pi):
    g = overflow_hub_graph()
    print(f"[parity] overflow hubs n={g.n} nnz={g.nnz} params {PARAM_SETS[pi]}", flush=True)
    res = L.Graph.from_csr(g).run(L.params(**PARAM_SETS[pi]))
    compare_run(res, O.run(g, oracle.Params(**PARAM_SETS[pi])), "overflow hubs")


@pytest.mark.parametrize("mode", ["0", "1", "2"])
def test_graph_capture_modes(L, O, mode, monkeypatch):
    """Colour-class iterations replayed from a captured HIP graph (mode 2),
    the default (mode 1) and no capture (mode 0) all give the oracle's run;
    each phase replays its graph once per iteration after the first, with the
    library's own synchronisations in between."""
    monkeypatch.setenv("LOUVAIN_HIP_GRAPHS", mode)
    p = dict(vf=1, color=1, color_cutoff=1)
    for g in (GG.rmat(13, 16, wmax=100, seed=6), hub_graph(seed=11, hub_deg=40000, extra=60000, n=50000)):
        print(f"[parity] graphs={mode} {g.name} n={g.n}", flush=True)
        res = L.Graph.from_csr(g).run(L.params(**p))
        compare_run(res, O.run(g, oracle.Params(**p)), f"graphs={mode} {g.name}")


@pytest.mark.parametrize("mode", ["0", "1"])
def test_rebuild_tile_sums_modes(L, O, mode, monkeypatch):
    """The rebuild with its pairs summed per tile before the sort (1) and with
    one key per entry (0) give the oracle's coarse graphs, step by step and
    over whole runs, for unit and weighted graphs."""
    monkeypatch.setenv("LOUVAIN_TILE_SUMS", mode)
    for g in (GG.sbm_1000(), GG.rmat(12, 8, seed=5), GG.rmat(13, 16, wmax=100, seed=6), hub_graph()):
        print(f"[parity] tile_sums={mode} {g.name} n={g.n}", flush=True)
        _steps(L, O, g, colored=False, vf=False, phases=3, iters=4)
        for d in (dict(), dict(vf=1, color=1, color_cutoff=1)):
            res = L.Graph.from_csr(g).run(L.params(**d))
            compare_run(res, O.run(g, oracle.Params(**d)), f"tile_sums={mode} {g.name} {d}")


def test_autotune_does_not_change_results(L, O, monkeypatch):
    """Lanes per vertex chosen by the tuner (a graph with bins above the
    tuning size) versus the defaults: identical runs, equal to the oracle."""
    g = GG.rmat(17, 16, seed=21)
    print(f"[parity] autotune {g.name} n={g.n} nnz={g.nnz}", flush=True)
    ref = O.run(g, oracle.Params())
    for mode in ("1", "0"):
        monkeypatch.setenv("LOUVAIN_AUTOTUNE", mode)
        res = L.Graph.from_csr(g).run(L.params())
        compare_run(res, ref, f"autotune={mode}")


@pytest.mark.parametrize("lanes", ["8,16,32,64,64,256", "4,4,8,16,32,64", "8,8,16,32,64,64"])
def test_fixed_lanes_equal_oracle(L, O, lanes, monkeypatch):
    """Every lanes-per-vertex choice the tuner may take gives the oracle's
    run (graphs with rows in bins 1..6, weighted, with self-loops)."""
    monkeypatch.setenv("LOUVAIN_LANES", lanes)
    for g in (GG.rmat(13, 16, wmax=100, seed=6), GG.chung_lu(20000, 2.1, 2000.0, 3.0e5, 150000, wmax=100, seed=4)):
        print(f"[parity] lanes={lanes} {g.name}", flush=True)
        res = L.Graph.from_csr(g).run(L.params(vf=1, color=1, color_cutoff=1))
        compare_run(res, O.run(g, oracle.Params(vf=1, color=1, color_cutoff=1)), f"lanes={lanes}")
        res = L.Graph.from_csr(g).run(L.params())
        compare_run(res, O.run(g, oracle.Params()), f"lanes={lanes} plain")


def spread_graph(base, starts, n):
    """base with gap isolated ids inserted before its vertex `at`, for each
    (at, gap) in starts, and isolated ids up to n after it: long runs of empty
    rows before, between and after the connected vertices, in the input and
    in every coarse graph."""
    newid = np.arange(base.n, dtype=np.int64)
    for at, gap in starts:
        newid[at:] += gap
    assert newid[-1] < n
    deg = np.diff(base.offsets)
    d = np.zeros(n, dtype=np.int64)
    d[newid] = deg
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum(d)
    g = SG.CSR(n, off, newid[base.cols].astype(np.int32), None if base.weights is None else base.weights.copy())
    g.name = f"spread({base.name}, n={n})"
    return g


def test_long_empty_row_gaps(L, O):
    """Degrees, colouring counts and coarse row offsets over long stretches
    of empty rows (isolated vertices before, between and after the connected
    ones)."""
    base = GG.rmat(12, 8, wmax=30, seed=13)
    g = spread_graph(base, [(0, 70000), (1000, 100000), (3000, 5)], base.n + 70000 + 100000 + 5 + 150000)
    _steps(L, O, g, colored=False, vf=True, phases=3, iters=4)
    _steps(L, O, g, colored=True, vf=False, phases=2, iters=3)
    for d in (dict(), dict(vf=1, color=1, color_cutoff=1000)):
        with L.Graph.from_csr(g) as gs:
            res = gs.run(L.params(**d))
        compare_run(res, O.run(g, oracle_params(d)), f"{g.name} {d}")


@pytest.mark.parametrize("case", range(3))
def test_plain_sweeps_above_one_launch_group(L, O, case):
    """Graphs of more than 65,536 vertices sweep through the separate small-
    and large-bin launches, where a plain sweep reads each neighbour's
    community together with that community's total (packed beside it before
    the sweep): unit and weighted R-MAT (scale 17) and a graph with a hub row
    of 20,000 entries, stepped iteration by iteration and run to the end."""
    g = [GG.rmat(17, 8, seed=7), GG.rmat(17, 8, wmax=100, seed=8),
         hub_graph(seed=13, hub_deg=20000, extra=100000, n=80000)][case]
    assert g.n > 65536
    _steps(L, O, g, colored=False, vf=(case == 1), phases=2, iters=4)
    with L.Graph.from_csr(g) as gs:
        gs.profile(True)
        res = gs.run(L.params())
        recs = {r["name"]: r for r in gs.profile_records()}
    compare_run(res, O.run(g, oracle_params(dict())), g.name)
    # every swept entry is charged to exactly one launch record
    assert sum(r["entries"] for n, r in recs.items() if n.startswith("sweep")) == \
        res.sweep_entries + res.lookahead_entries
    assert recs["sweep_pack_communities"]["launches"] > 0


def test_gain_bound_cases(L, O):
    """The best community need not be one of the largest edge weight: vertex 0
    (self-loop 10) has weight 3 to the heavy star centre 1 and weight 1 to the
    light vertex 2, and G(2) > G(1) in the first sweep; the graph is also
    repeated with its ids reversed (the singlet rule then lets 0 move)."""
    edges = [(0, 0), (0, 1), (0, 2), (2, 8)] + [(1, v) for v in range(3, 8)]
    w = [10, 3, 1, 1] + [2] * 5
    g = SG.from_edges(9, edges, w, name="gain_bound")
    r = SG.from_edges(9, [(8 - u, 8 - v) if u >= v else (8 - v, 8 - u) for u, v in edges], w, name="gain_bound_rev")
    for x in (g, r):
        _steps(L, O, x, colored=False, vf=False, phases=2, iters=3)
        for d in (dict(), dict(singlet_rule=0)):
            compare_run(L.Graph.from_csr(x).run(L.params(**d)), O.run(x, oracle_params(d)), f"{x.name} {d}")


def heavy_graph(seed, n, extra, hub_deg, name):
    """Weights uniform in [2^30, 2^31 - 1]: 2m * k_max is far above 2^62, so
    gains take the 128-bit path and the LDS sums the 64-bit one (vertex 0 is
    a hub of hub_deg neighbours when hub_deg > 0)."""
    rng = np.random.default_rng(seed)
    edges = set()
    if hub_deg:
        for v in rng.choice(np.arange(1, n), size=hub_deg, replace=False):
            edges.add((0, int(v)))
    while len(edges) < hub_deg + extra:
        u, v = (int(x) for x in rng.integers(0, n, 2))
        if u != v:
            edges.add((min(u, v), max(u, v)))
    edges = sorted(edges)
    w = rng.integers(1 << 30, (1 << 31) - 1, size=len(edges))
    return SG.from_edges(n, edges, w, name=name)


def test_wide_gains(L, O):
    """The 128-bit gain path (2m * k_max >= 2^62) of every kernel that
    evaluates gains: the binned sweep, both hub passes, the hub decision of
    the plain and the coloured commit, and the batched form."""
    gs = [heavy_graph(5, 60, 300, 0, "heavy_small"), heavy_graph(6, 6000, 20000, 3000, "heavy_hub")]
    for g in gs:
        with L.Graph.from_csr(g) as h:
            info = h.info()
        assert info["two_m"] * info["k_max"] >= 1 << 62 and info["two_m"] < 1 << 62, g.name
        _steps(L, O, g, colored=False, vf=True, phases=2, iters=3)
        _steps(L, O, g, colored=True, vf=False, phases=2, iters=3)
        for d in (dict(), dict(vf=1, color=1, color_cutoff=10)):
            with L.Graph.from_csr(g) as h:
                res = h.run(L.params(**d))
            compare_run(res, O.run(g, oracle_params(d)), f"{g.name} {d}")
    b = L.Batch.from_graphs(gs)
    res = b.run(L.params())
    b.close()
    for g, r in zip(gs, res):
        ref = O.run(g, oracle.Params())
        assert np.array_equal(r.labels, ref.labels) and (r.N, r.D) == (ref.N, ref.D), g.name


def test_vf_rebuild_cases(L, O):
    """The vertex-following rebuild on a graph with every case: a kept vertex
    with a self-loop and two absorbed leaves, a leaf on another kept vertex,
    an isolated pair, an isolated vertex, a vertex whose only entry is a
    self-loop, and a chain (a degree-1 end on a degree-2 vertex)."""
    edges = [(0, 0), (0, 1), (0, 2), (0, 3), (3, 4), (5, 6), (8, 8), (3, 9), (9, 10), (10, 11), (11, 12)]
    w = [5, 3, 4, 2, 1, 7, 9, 1, 2, 6, 8]
    g = SG.from_edges(14, edges, w, name="vf_cases")
    _steps(L, O, g, colored=False, vf=True, phases=2, iters=3)
    for d in (dict(vf=1), dict(vf=1, color=1, color_cutoff=1), dict(vf=1, singlet_rule=0)):
        with L.Graph.from_csr(g) as h:
            res = h.run(L.params(**d))
        compare_run(res, O.run(g, oracle_params(d)), f"vf_cases {d}")
