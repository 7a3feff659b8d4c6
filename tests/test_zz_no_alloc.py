"""The allocation-free entry point (louvain_run_noalloc) against the
allocating one (louvain_init_csr + louvain_run) through the C ABI: two calls
in a row on the shared device scratch, the second on a smaller graph, each
equal bit for bit to the ordinary run; and the size limit refused up front."""
import ctypes

import numpy as np
import pytest

import small_graphs as SG
from paper_1410_1237_amd import graphs as GG


def _lib():
    from paper_1410_1237_amd import louvain
    louvain.lib()
    return louvain


def test_noalloc_refuses_oversized_graph():
    L = _lib()
    # sizes only: the check runs before any device work, so no pointer is read
    fake = ctypes.c_void_p(0x1000)
    with pytest.raises(L.LouvainError) as e:
        L.louvain_run_noalloc(1 << 20, 1 << 24, fake.value, fake.value, None, L.params(), hip_stream=0)
    assert e.value.status == L.E_INVALID_ARG
    assert "too large" in str(e.value)


def _device(g):
    import torch
    dev = torch.device("cuda:0")
    off = torch.from_numpy(np.ascontiguousarray(g.offsets, dtype=np.int64)).to(dev)
    col = torch.from_numpy(np.ascontiguousarray(g.cols, dtype=np.int32)).to(dev)
    w = None if g.weights is None else torch.from_numpy(np.ascontiguousarray(g.weights, dtype=np.int32)).to(dev)
    return off, col, w


def _phases(res):
    out = []
    for p in range(res.phases):
        ph = res.phase[p]
        its = [res.iter[ph.first_iter + t] for t in range(ph.iterations)]
        out.append((ph.n, ph.nnz, ph.colored, ph.num_colors, ph.iterations, ph.hit_max_iter, ph.loss_undone,
                    ph.q_num.value(), [(it.moves, it.q_num.value()) for it in its]))
    return out


@pytest.mark.gpu
def test_noalloc_equals_allocating_run_twice():
    import torch
    assert torch.cuda.is_available()
    L = _lib()
    cases = [(GG.rmat(13, 16, wmax=100, seed=6), dict(vf=1, color=1, color_cutoff=1000)),
             (GG.sbm_1000(), dict()),
             (SG.star(3000), dict(vf=1))]
    for g, d in cases:
        print(f"[noalloc] {g.name} n={g.n} nnz={g.nnz} {d}", flush=True)
        p = L.params(**d)
        off, col, w = _device(g)
        # the ordinary entry points
        h = L.louvain_init_csr(g.n, g.nnz, off.data_ptr(), col.data_ptr(), None if w is None else w.data_ptr(),
                               L.DEVICE_PTRS)
        lab_ref = torch.empty(g.n, dtype=torch.int32, device="cuda:0")
        ref = L.louvain_run(h, p, lab_ref.data_ptr(), 1)
        ref_phases = _phases(ref)
        ref_sc = (ref.num_communities, ref.q_num.value(), ref.q_den.value(), ref.q0_num.value(), ref.q, ref.n_vf)
        L.louvain_destroy(h)
        # the allocation-free one
        lab = torch.full((g.n,), -1, dtype=torch.int32, device="cuda:0")
        res = L.louvain_run_noalloc(g.n, g.nnz, off.data_ptr(), col.data_ptr(),
                                    None if w is None else w.data_ptr(), p, lab.data_ptr(), L.VALIDATE)
        torch.cuda.synchronize()
        sc = (res.num_communities, res.q_num.value(), res.q_den.value(), res.q0_num.value(), res.q, res.n_vf)
        assert sc == ref_sc
        assert _phases(res) == ref_phases
        assert torch.equal(lab, lab_ref)
