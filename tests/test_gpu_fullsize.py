"""Full-size parity: the library on the full synthetic workloads, in the
configuration the benchmark times (CSR already on the device, labels written
to device memory), against stored oracle results (tests/golden, written by
make_golden.py from the oracle alone), and sampled first-sweep decisions of
R-MAT scale 24 against the oracle computed vertex by vertex."""
import glob
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_1410_1237_amd import graphs as GG

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
# single-workload records (the per-graph records of the mixes are checked by test_gpu_mixes.py)
GOLDEN = sorted(p for p in glob.glob(os.path.join(HERE, "golden", "*.json")) if "_x" not in os.path.basename(p))
HEUR = {"plain": {}, "full": {"vf": 1, "color": 1}}


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available()
    from paper_1410_1237_amd import louvain
    louvain.lib()
    return louvain


_graphs = {}


def workload(name):
    if name not in _graphs:
        _graphs.clear()  # keep one large graph in host memory at a time
        _graphs[name] = GG.WORKLOADS[name]()
    return _graphs[name]


@pytest.mark.parametrize("path", GOLDEN, ids=[os.path.basename(p)[:-5] for p in GOLDEN])
def test_full_run_equals_oracle_golden(L, path):
    import torch
    with open(path) as f:
        ref = json.load(f)
    g = workload(ref["workload"])
    print(f"[fullsize] {ref['workload']} {ref['heuristics']} n={g.n} nnz={g.nnz}", flush=True)
    assert (g.n, g.nnz) == (ref["n"], ref["nnz"])
    dev = torch.device("cuda:0")
    off = torch.from_numpy(g.offsets).to(dev)
    col = torch.from_numpy(g.cols).to(dev)
    w = torch.from_numpy(g.weights).to(dev) if g.weights is not None else None
    labels = torch.empty(g.n, dtype=torch.int32, device=dev)
    h = L.Graph.from_tensors(off, col, w, validate=False)
    r = h.run(L.params(**HEUR[ref["heuristics"]]), labels=labels)
    h.close()
    lab = labels.cpu().numpy().astype("<i4")
    assert (r.K, r.N, r.D, r.n_vf, r.N0) == (ref["K"], int(ref["N"]), int(ref["D"]), ref["n_vf"], int(ref["N0"]))
    assert r.q == ref["q"]
    assert len(r.phases) == len(ref["phases"])
    for a, b in zip(r.phases, ref["phases"]):
        assert (a.n, a.nnz, a.colored, a.num_colors, a.iterations) == \
               (b["n"], b["nnz"], b["colored"], b["ncolors"], b["iterations"])
        assert a.moves == b["moves"]
        assert [str(x) for x in a.N_iter] == b["N_iter"] and str(a.N_end) == b["N_end"]
        assert a.undone == b["undone"]
    assert hashlib.sha256(lab.tobytes()).hexdigest() == ref["labels_sha256"]


def test_rmat24_first_sweep_sampled(L):
    """Decisions of the first synchronous sweep of R-MAT scale 24 (all
    singletons): every hub with more than 2,048 entries plus 3,000 seeded
    random vertices, each recomputed by the oracle."""
    import torch
    g = workload("rmat_s24")
    dev = torch.device("cuda:0")
    off = torch.from_numpy(g.offsets).to(dev)
    col = torch.from_numpy(g.cols).to(dev)
    h = L.Graph.from_tensors(off, col, None, validate=False)
    s = h.sweep(L.params())
    comm = h.state()["comm"]
    h.close()
    deg = np.diff(g.offsets)
    rng = np.random.default_rng(24)
    sample = np.unique(np.concatenate([np.nonzero(deg > 2048)[0], rng.integers(0, g.n, 3000)]))
    st = oracle.default().state(g)
    got = comm[sample]
    want = np.array([st.decide(int(i)) for i in sample], dtype=np.int32)
    assert np.array_equal(got, want)
    assert s["entries"] == g.nnz
