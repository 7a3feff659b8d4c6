"""Served form: jobs submitted while others run are admitted into batches as
slots and budget free up, and every job's result is the one it gets alone
(and, for small jobs, the oracle's)."""
import time

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


def job_mix():
    rng = np.random.default_rng(91)
    gs = [GG.batch_sbm(i) for i in range(100, 120)]
    gs += [GG.served_job(i) for i in range(12) if GG.served_job_params(i)["n"] <= 300_000]
    gs += [SG.random_graph(rng, int(rng.integers(5, 40)), p=0.3, self_loops=0.3, wmax=7) for _ in range(4)]
    gs += [SG.from_edges(0, []), SG.from_edges(2, [(0, 1)]), SG.star(25)]
    rng.shuffle(gs)
    return gs


def solo(L, g, p):
    h = L.Graph.from_csr(g)
    r = h.run(p)
    h.close()
    return r


def check_job(L, O, g, info, ref, tag):
    assert info.status == L.OK, tag
    assert np.array_equal(info.labels, ref.labels), tag + ": labels"
    assert (info.K, info.N, info.D, info.q, info.n_vf) == (ref.K, ref.N, ref.D, ref.q, ref.n_vf), tag
    assert info.phases == len(ref.phases), tag
    assert info.t_submit <= info.t_admit <= info.t_done, tag
    if g.n <= 3000:
        o = O.run(g, oracle.Params())
        assert np.array_equal(info.labels, o.labels) and (info.N, info.D) == (o.N, o.D), tag + ": oracle"


@pytest.mark.parametrize("inflight,per_batch", [(3, 5), (1, 64)])
def test_served_mix_equals_alone(L, O, inflight, per_batch):
    gs = job_mix()
    print(f"[serve] {len(gs)} jobs, inflight {inflight}, per batch {per_batch}", flush=True)
    p = L.params()
    refs = [solo(L, g, p) for g in gs]
    s = L.Server(p, max_inflight_batches=inflight, max_batch_graphs=per_batch)
    tickets = []
    for i, g in enumerate(gs):  # staggered arrivals: later jobs come while earlier ones run
        tickets.append(s.submit(g))
        if i % 7 == 6:
            time.sleep(0.01)
    s.wait_all()
    infos = [s.poll(t) for t in tickets]
    for g, info, ref in zip(gs, infos, refs):
        check_job(L, O, g, info, ref, g.name)
    batches = {i.batch_id for i in infos}
    assert len(batches) >= -(-len(gs) // per_batch)
    assert all(i.batch_graphs <= per_batch for i in infos)
    for t in tickets:
        s.release(t)
    s.close()


def test_served_solo_and_borrowed(L, O):
    """Jobs above the size threshold run alone through the single-graph path,
    the rest in batches; borrowed submissions (no copy) give the same results."""
    gs = job_mix()
    p = L.params()
    refs = [solo(L, g, p) for g in gs]
    s = L.Server(p, max_inflight_batches=3, max_batch_graphs=16, solo_min_vertices=20000)
    tickets = [s.submit(g, borrow=(i % 2 == 0)) for i, g in enumerate(gs)]
    s.wait_all()
    infos = [s.poll(t) for t in tickets]
    for g, info, ref in zip(gs, infos, refs):
        check_job(L, O, g, info, ref, g.name)
        if g.n >= 20000:
            assert info.batch_graphs == 1, g.name
    assert any(i.batch_graphs > 1 for i in infos)
    s.close()


def job_bytes(g):
    # the server's estimate of a job's device footprint
    big = max(g.n, g.nnz) + 1
    return 24 * (g.n + 1) + 32 * g.nnz + 40 * big + 120 * g.n


def test_served_budget(L, O):
    gs = [GG.batch_sbm(i) for i in range(120, 140)]
    sizes = sorted(job_bytes(g) for g in gs)
    budget = sizes[-1] + sizes[-2] + sizes[-3]  # about three of these jobs at a time
    big = GG.rmat(18, 16, seed=9)
    assert job_bytes(big) > budget
    p = L.params()
    s = L.Server(p, hbm_budget_bytes=budget, max_inflight_batches=4)
    tickets = [s.submit(g) for g in gs]
    tb = s.submit(big)
    s.wait_all()
    infos = [s.poll(t) for t in tickets]
    for g, info in zip(gs, infos):
        check_job(L, O, g, info, solo(L, g, p), g.name)
    assert len({i.batch_id for i in infos}) >= -(-sum(sizes) // budget)
    assert s.poll(tb).status == L.E_OOM
    s.close()


def test_served_rejects(L):
    with pytest.raises(L.LouvainError):
        L.Server(L.params(color=1))
    s = L.Server(L.params())
    bad = SG.from_edges(3, [(0, 1)])
    bad.cols = bad.cols.copy()
    bad.cols[0] = 7
    with pytest.raises(L.LouvainError):
        s.submit(bad)
    t = s.submit(SG.from_edges(2, [(0, 1)]))
    s.wait_all()
    info = s.poll(t)
    assert info.status == L.OK and info.K == 1
    s.release(t)
    with pytest.raises(L.LouvainError):
        s.poll(t)
    s.close()


def test_served_invalid_job_fails_alone(L, O):
    """A job that passes the submit checks but not the device validation
    (an asymmetric CSR) fails with LOUVAIN_E_BAD_CSR; the jobs batched with it
    still get their own results."""
    good = [GG.batch_sbm(i) for i in range(140, 146)]
    bad = SG.from_edges(4, [(0, 1), (1, 2), (2, 3)])
    bad.cols = bad.cols.copy()
    bad.cols[0] = 2  # row 0 now points to 2, but row 2 has no entry back to 0
    # borrowed: not range-checked at submission, the device validation rejects it
    far = SG.from_edges(4, [(0, 1), (1, 2), (2, 3)])
    far.cols = far.cols.copy()
    far.cols[0] = 9
    p = L.params()
    s = L.Server(p, max_inflight_batches=1, max_batch_graphs=8)
    tickets = [s.submit(g) for g in good[:3]] + [s.submit(bad), s.submit(far, borrow=True)] + \
        [s.submit(g, borrow=True) for g in good[3:]]
    s.wait_all()
    infos = [s.poll(t) for t in tickets]
    assert infos[3].status == L.E_BAD_CSR and infos[4].status == L.E_BAD_CSR
    for g, info in zip(good, infos[:3] + infos[5:]):
        check_job(L, O, g, info, solo(L, g, p), g.name)
    s.close()


def test_served_invalid_large_job(L, O):
    """A job large enough to run alone that fails the device validation fails
    with LOUVAIN_E_BAD_CSR; the server keeps serving."""
    big = GG.batch_sbm(150)
    assert big.n >= 2000
    bad = SG.CSR(big.n, big.offsets.copy(), big.cols.copy(), None if big.weights is None else big.weights.copy())
    bad.name = "asym"
    row0 = slice(int(bad.offsets[0]), int(bad.offsets[1]))
    bad.cols[row0] = np.sort((bad.cols[row0] + 1) % bad.n)  # row 0's entries lose their mirrors
    p = L.params()
    s = L.Server(p, solo_min_vertices=1000)
    t_bad = s.submit(bad, borrow=True)
    t_ok = s.submit(big)
    s.wait_all()
    assert s.poll(t_bad).status == L.E_BAD_CSR
    info = s.poll(t_ok)
    check_job(L, O, big, info, solo(L, big, p), big.name)
    assert info.batch_graphs == 1
    s.close()
