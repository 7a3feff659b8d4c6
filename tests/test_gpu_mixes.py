"""The batched and served workloads at full size against the oracle's stored
per-graph results (tests/golden/*_x*_plain.json, written by make_golden.py
from the oracle alone): every one of the 4,096 SBMs of the batched mix in one
batched run, and every job of the served mix (1e3 to 2e6 vertices) through
the request loop with its jobs submitted at once; K, the exact modularity
pair and the SHA-256 of the labels of each graph."""
import concurrent.futures as cf
import hashlib
import json
import os

import numpy as np
import pytest

from paper_1410_1237_amd import graphs as GG

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available()
    from paper_1410_1237_amd import louvain
    louvain.lib()
    return louvain


def golden(mix, count):
    path = os.path.join(HERE, "golden", f"{mix}_x{count}_plain.json")
    with open(path) as f:
        data = json.load(f)
    return {r[0]: r for r in data["graphs"]}


def sha16(labels):
    return hashlib.sha256(np.ascontiguousarray(labels, dtype="<i4").tobytes()).hexdigest()[:16]


def generate(fn, count):
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(fn, range(count)))


def test_batched_4096_sbms_equal_oracle(L):
    import torch
    ref = golden("batch_sbm", 4096)
    gs = generate(GG.batch_sbm, 4096)
    goff, off, col, w = L.union_csr(gs)
    print(f"[mix] batched: {len(gs)} graphs n={int(goff[-1])} nnz={len(col)}", flush=True)
    dev = torch.device("cuda:0")
    labels = torch.empty(int(goff[-1]), dtype=torch.int32, device=dev)
    b = L.Batch.from_union(goff, torch.from_numpy(off).to(dev), torch.from_numpy(col).to(dev),
                           torch.from_numpy(w).to(dev) if w is not None else None)
    res = b.run(L.params(), labels=labels, stats=False)
    b.close()
    lab = labels.cpu().numpy()
    bad = []
    for i, (g, r) in enumerate(zip(gs, res)):
        rec = ref[i]
        got = (g.n, g.nnz, r.K, str(r.N), str(r.D), sha16(lab[goff[i]:goff[i + 1]]))
        want = (rec[1], rec[2], rec[3], rec[4], rec[5], rec[8])
        if got != want:
            bad.append((i, got, want))
    assert not bad, f"{len(bad)} graphs differ from the oracle, first: {bad[:3]}"


def test_served_mix_equals_oracle(L):
    ref = golden("served", 128)
    jobs = generate(GG.served_job, 128)
    print(f"[mix] served: {len(jobs)} jobs n={sum(g.n for g in jobs)} nnz={sum(g.nnz for g in jobs)}", flush=True)
    s = L.Server(L.params())
    tickets = [s.submit(g, borrow=True) for g in jobs]
    s.wait_all()
    infos = [s.poll(t, labels=True) for t in tickets]
    s.close()
    bad = []
    for j, (g, inf) in enumerate(zip(jobs, infos)):
        rec = ref[j]
        got = (inf.status, g.n, g.nnz, inf.K, str(inf.N), str(inf.D), sha16(inf.labels))
        want = (L.OK, rec[1], rec[2], rec[3], rec[4], rec[5], rec[8])
        if got != want:
            bad.append((j, got, want))
    assert not bad, f"{len(bad)} jobs differ from the oracle, first: {bad[:3]}"
