"""Batched form: every graph of a batch gets exactly its oracle result
(labels, K, exact modularity, per-phase and per-iteration statistics), for
graphs of uneven sizes, with hubs, self-loops, weights and degenerate cases,
under several parameter sets."""
import numpy as np
import pytest

import oracle
import small_graphs as SG
from paper_1410_1237_amd import graphs as GG
from test_gpu_parity import compare_run, hub_graph

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


def mixed_graphs():
    rng = np.random.default_rng(77)
    gs = [GG.batch_sbm(i) for i in range(12)]
    gs += [SG.random_graph(rng, int(rng.integers(5, 40)), p=0.3, self_loops=0.3, wmax=7) for _ in range(6)]
    gs += [SG.from_edges(0, []), SG.from_edges(3, []), SG.from_edges(2, [(0, 1)]), SG.star(30),
           SG.ring_of_cliques(5, 4), hub_graph(), GG.rmat(11, 16, seed=8)]
    rng.shuffle(gs)
    return gs


PARAMS = [dict(), dict(vf=1), dict(singlet_rule=0), dict(max_iter=3, max_phases=2),
          dict(threshold_mode=1, theta_final=(1, 10000)), dict(vf=2)]


@pytest.mark.parametrize("pi", range(len(PARAMS)))
def test_batch_equals_oracle(L, O, pi):
    gs = mixed_graphs()
    print(f"[batch] {len(gs)} graphs, params {PARAMS[pi]}", flush=True)
    b = L.Batch(gs)
    res = b.run(L.params(**PARAMS[pi]))
    b.close()
    for g, r in zip(gs, res):
        compare_run(r, O.run(g, oracle.Params(**PARAMS[pi])), f"{g.name} {PARAMS[pi]}")


def test_batch_equals_solo_runs(L):
    gs = [GG.batch_sbm(i) for i in range(30, 60)]
    b = L.Batch(gs)
    res = b.run(L.params())
    res2 = b.run(L.params())
    b.close()
    for g, r, r2 in zip(gs, res, res2):
        solo = L.Graph.from_csr(g).run(L.params())
        assert np.array_equal(r.labels, solo.labels) and np.array_equal(r.labels, r2.labels)
        assert (r.N, r.D, r.K, r.q) == (solo.N, solo.D, solo.K, solo.q)
        assert [p.moves for p in r.phases] == [p.moves for p in solo.phases]


def test_batch_order_invariance(L):
    gs = [GG.batch_sbm(i) for i in range(60, 80)]
    a = L.Batch(gs).run(L.params(), stats=False)
    perm = list(reversed(range(len(gs))))
    b = L.Batch([gs[i] for i in perm]).run(L.params(), stats=False)
    for j, i in enumerate(perm):
        assert np.array_equal(a[i].labels, b[j].labels) and a[i].N == b[j].N


def test_batch_rejects(L):
    g1, g2 = SG.from_edges(2, [(0, 1)]), SG.from_edges(2, [(0, 1)])
    goff, off, col, w = L.union_csr([g1, g2])
    col = col.copy()
    col[0] = 2  # an edge into the other graph (and asymmetric)
    with pytest.raises(L.LouvainError):
        L.louvain_batch_init(2, goff, len(col), off, col, None, 0)
    b = L.Batch([g1, g2])
    with pytest.raises(L.LouvainError):
        b.run(L.params(color=1))
    b.close()


def test_batch_from_separate_graphs(L, O):
    """louvain_batch_init_graphs (per-graph host arrays packed on the device)
    gives the same runs as the union path and the oracle, with empty graphs,
    unweighted graphs among weighted ones and hubs."""
    gs = mixed_graphs()
    b1 = L.Batch.from_graphs(gs)
    r1 = b1.run(L.params())
    b1.close()
    b2 = L.Batch(gs)
    r2 = b2.run(L.params())
    b2.close()
    for g, x, y in zip(gs, r1, r2):
        assert np.array_equal(x.labels, y.labels) and (x.N, x.D, x.K) == (y.N, y.D, y.K), g.name
        compare_run(x, O.run(g, oracle.Params()), g.name)
