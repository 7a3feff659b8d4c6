"""Host-side checks of the C-ABI library that need no GPU: it loads, and it
exports every entry point declared in include/louvain.h."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "louvain.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(louvain_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_boundary():
    names = declared()
    for n in ["louvain_init_csr", "louvain_color", "louvain_sweep", "louvain_coarsen", "louvain_run",
              "louvain_vf", "louvain_destroy", "louvain_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1410_1237_amd import louvain as L
    lib = L.lib()
    for name in declared():
        assert hasattr(lib, name), name
    assert sorted(L.EXPORTS) == sorted(declared())


def test_params_defaults_without_gpu():
    from paper_1410_1237_amd import louvain as L
    p = L.params()
    assert (p.singlet_rule, p.vf, p.color, p.max_iter, p.max_phases) == (1, 0, 0, 1000, 100)
    assert (p.theta_color.num, p.theta_color.den) == (1, 100)
    assert (p.theta_final.num, p.theta_final.den) == (1, 1000000)
    assert p.color_cutoff == 100000 and p.color_seed == 0x4C4F5556


def test_init_rejects_bad_arguments_on_host():
    # rejected before any device work, so these run without a GPU
    import numpy as np
    from paper_1410_1237_amd import louvain as L
    off = np.array([0, 1, 2], dtype=np.int64)
    col = np.array([1, 0], dtype=np.int32)
    with pytest.raises(L.LouvainError) as e:
        L.louvain_init_csr(-1, 2, off, col)
    assert e.value.status == L.E_INVALID_ARG
    bad = np.array([0, 1, 3], dtype=np.int64)
    with pytest.raises(L.LouvainError) as e:
        L.louvain_init_csr(2, 2, bad, col)
    assert e.value.status == L.E_BAD_CSR
    assert "offsets" in L.louvain_last_error(None)


def test_no_oracle_on_product_path():
    # the product package never imports the oracle
    pkg = os.path.join(ROOT, "paper_1410_1237_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".c", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "liboracle" not in src, f


def test_server_config_and_host_rejection():
    from paper_1410_1237_amd import louvain as L
    c = L.louvain_server_config_default()
    assert c.hbm_budget_bytes == 200 << 30 and c.max_inflight_batches == 4
    assert c.max_batch_graphs == 4096 and c.max_batch_vertices == 0 and c.solo_min_vertices == 100000
    with pytest.raises(L.LouvainError) as e:  # colored mode is not served
        L.Server(L.params(color=1))
    assert e.value.status == L.E_INVALID_ARG
    with pytest.raises(L.LouvainError) as e:
        L.Server(L.params(), max_inflight_batches=0)
    assert e.value.status == L.E_INVALID_ARG
    with pytest.raises(L.LouvainError) as e:
        L.Server(L.params(), solo_min_vertices=-1)
    assert e.value.status == L.E_INVALID_ARG


def test_library_has_no_undefined_internal_symbols():
    # every internal routine the library calls is defined in it (a missing
    # template instance would only fail when the library is loaded)
    import subprocess
    from paper_1410_1237_amd import louvain as L
    out = subprocess.run(["nm", "-C", "--undefined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    assert "lv::" not in out, out


def test_batch_init_graphs_host_rejection():
    # rejected on the host before any device call
    import ctypes
    import numpy as np
    from paper_1410_1237_amd import louvain as L
    off = np.array([1, 2], dtype=np.int64)  # must start at 0
    col = np.array([0], dtype=np.int32)
    n = np.array([1], dtype=np.int64)
    nnz = np.array([1], dtype=np.int64)
    P = ctypes.c_void_p * 1
    h = ctypes.c_void_p()
    st = L.lib().louvain_batch_init_graphs(1, n.ctypes.data, nnz.ctypes.data, P(off.ctypes.data), P(col.ctypes.data),
                                           None, 0, None, ctypes.byref(h))
    assert st == L.E_BAD_CSR
    st = L.lib().louvain_batch_init_graphs(1, n.ctypes.data, nnz.ctypes.data, P(off.ctypes.data), P(col.ctypes.data),
                                           None, L.DEVICE_PTRS, None, ctypes.byref(h))
    assert st == L.E_INVALID_ARG
