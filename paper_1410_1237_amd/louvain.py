"""Thin ctypes binding of liblouvain.so (C ABI in include/louvain.h).

Argument marshalling only: every step runs in the library's HIP kernels.
Functions carry the C names (``louvain_init_csr``, ``louvain_vf``,
``louvain_color``, ``louvain_sweep``, ``louvain_coarsen``, ``louvain_run``,
...); ``Graph`` bundles them around one handle.  PyTorch is used only for
device buffers and the current HIP stream.  There is no fallback: if the
library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblouvain.so")

OK, E_INVALID_ARG, E_BAD_CSR, E_OOM, E_HIP, E_OVERFLOW, E_STATE = range(7)
DEVICE_PTRS = 1
VALIDATE = 2
DEFAULT_SEED = 0x4C4F5556


class LouvainError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"louvain status {status}: {msg}")
        self.status = status


class Ratio(ctypes.Structure):
    _fields_ = [("num", ctypes.c_int64), ("den", ctypes.c_int64)]


class I128(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_int64)]

    def value(self) -> int:
        return (int(self.hi) << 64) | int(self.lo)


class Params(ctypes.Structure):
    _fields_ = [("vf", ctypes.c_int32), ("color", ctypes.c_int32), ("singlet_rule", ctypes.c_int32),
                ("threshold_mode", ctypes.c_int32), ("color_first_phase_only", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("max_phases", ctypes.c_int32), ("color_balance", ctypes.c_int32),
                ("theta_color", Ratio), ("theta_final", Ratio), ("color_cutoff", ctypes.c_int64),
                ("color_seed", ctypes.c_uint64)]


class IterStats(ctypes.Structure):
    _fields_ = [("moves", ctypes.c_int64), ("q_num", I128), ("pairs", ctypes.c_int64),
                ("entries", ctypes.c_int64), ("ms", ctypes.c_float), ("reserved", ctypes.c_int32)]


class PhaseStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("colored", ctypes.c_int32),
                ("num_colors", ctypes.c_int32), ("iterations", ctypes.c_int32), ("hit_max_iter", ctypes.c_int32),
                ("loss_undone", ctypes.c_int32), ("reserved", ctypes.c_int32), ("first_iter", ctypes.c_int64), ("q_num", I128), ("ms_color", ctypes.c_double),
                ("ms_sweep", ctypes.c_double), ("ms_coarsen", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("n_orig", ctypes.c_int64), ("n_vf", ctypes.c_int64), ("num_communities", ctypes.c_int64),
                ("phases", ctypes.c_int64), ("iterations", ctypes.c_int64), ("q_num", I128), ("q_den", I128),
                ("q0_num", I128), ("q", ctypes.c_double), ("sweep_entries", ctypes.c_int64),
                ("lookahead_entries", ctypes.c_int64), ("vf_rounds", ctypes.c_int64), ("ms_total", ctypes.c_double), ("ms_vf", ctypes.c_double), ("ms_color", ctypes.c_double),
                ("ms_sweep", ctypes.c_double), ("ms_coarsen", ctypes.c_double),
                ("phase", ctypes.POINTER(PhaseStats)), ("iter", ctypes.POINTER(IterStats))]


class GraphResult(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("num_communities", ctypes.c_int64),
                ("phases", ctypes.c_int64), ("iterations", ctypes.c_int64), ("q_num", I128), ("q_den", I128),
                ("q0_num", I128), ("q", ctypes.c_double), ("n_vf", ctypes.c_int64)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_inflight_batches", ctypes.c_int32),
                ("max_batch_graphs", ctypes.c_int32), ("max_batch_vertices", ctypes.c_int64),
                ("solo_min_vertices", ctypes.c_int64)]


class JobResult(ctypes.Structure):
    _fields_ = [("result", GraphResult), ("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("batch_id", ctypes.c_int64), ("batch_graphs", ctypes.c_int64), ("t_packed", ctypes.c_double),
                ("t_ready", ctypes.c_double)]


_lib = None

EXPORTS = ["louvain_params_default", "louvain_init_csr", "louvain_vf", "louvain_color", "louvain_sweep",
           "louvain_coarsen", "louvain_run", "louvain_destroy", "louvain_last_error", "louvain_get_info",
           "louvain_get_state", "louvain_get_graph", "louvain_get_colors", "louvain_get_map", "louvain_profile",
           "louvain_profile_get", "louvain_batch_init", "louvain_batch_run", "louvain_batch_graph_stats",
           "louvain_batch_destroy", "louvain_batch_last_error", "louvain_batch_init_graphs",
           "louvain_server_config_default",
           "louvain_server_create", "louvain_server_submit", "louvain_server_submit_borrowed",
           "louvain_server_poll", "louvain_server_release",
           "louvain_server_wait_all", "louvain_server_last_error", "louvain_server_destroy",
           "louvain_run_noalloc", "louvain_vf_chain", "louvain_color_balance"]


def lib():
    """The loaded library; raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1410_1237_amd.build`")
    # torch ships its own HIP runtime under the same soname: load it first so
    # that the library binds to that one instead of bringing a second runtime
    # into the process (the second to initialise finds no device)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
    st = ctypes.c_int
    L.louvain_params_default.argtypes = [ctypes.POINTER(Params)]
    L.louvain_params_default.restype = None
    L.louvain_init_csr.argtypes = [i64, i64, vp, vp, vp, u32, vp, ctypes.POINTER(vp)]
    L.louvain_init_csr.restype = st
    L.louvain_vf.argtypes = [vp, ctypes.POINTER(i64)]
    L.louvain_vf.restype = st
    L.louvain_vf_chain.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.louvain_vf_chain.restype = st
    L.louvain_color.argtypes = [vp, u64, ctypes.POINTER(i32)]
    L.louvain_color.restype = st
    L.louvain_color_balance.argtypes = [vp, u64, ctypes.POINTER(i64)]
    L.louvain_color_balance.restype = st
    L.louvain_sweep.argtypes = [vp, ctypes.POINTER(Params), ctypes.POINTER(IterStats)]
    L.louvain_sweep.restype = st
    L.louvain_coarsen.argtypes = [vp, ctypes.POINTER(i64)]
    L.louvain_coarsen.restype = st
    L.louvain_run.argtypes = [vp, ctypes.POINTER(Params), vp, u32, ctypes.POINTER(Result)]
    L.louvain_run.restype = st
    L.louvain_run_noalloc.argtypes = [i64, i64, vp, vp, vp, u32, ctypes.POINTER(Params), vp, vp,
                                      ctypes.POINTER(Result)]
    L.louvain_run_noalloc.restype = st
    L.louvain_destroy.argtypes = [vp]
    L.louvain_destroy.restype = None
    L.louvain_last_error.argtypes = [vp]
    L.louvain_last_error.restype = ctypes.c_char_p
    L.louvain_get_info.argtypes = [vp, vp]
    L.louvain_get_info.restype = st
    L.louvain_get_state.argtypes = [vp, vp, vp, vp, vp, u32]
    L.louvain_get_state.restype = st
    L.louvain_get_graph.argtypes = [vp, vp, vp, vp, u32]
    L.louvain_get_graph.restype = st
    L.louvain_get_colors.argtypes = [vp, vp, u32]
    L.louvain_get_colors.restype = st
    L.louvain_get_map.argtypes = [vp, vp, u32]
    L.louvain_get_map.restype = st
    L.louvain_profile.argtypes = [vp, i32]
    L.louvain_profile.restype = st
    L.louvain_profile_get.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(i64),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]
    L.louvain_profile_get.restype = st
    L.louvain_batch_init.argtypes = [i32, vp, i64, vp, vp, vp, u32, vp, ctypes.POINTER(vp)]
    L.louvain_batch_init.restype = st
    L.louvain_batch_run.argtypes = [vp, ctypes.POINTER(Params), vp, u32, vp]
    L.louvain_batch_run.restype = st
    L.louvain_batch_graph_stats.argtypes = [vp, i32, ctypes.POINTER(ctypes.POINTER(PhaseStats)),
                                            ctypes.POINTER(i64), ctypes.POINTER(ctypes.POINTER(IterStats)),
                                            ctypes.POINTER(i64)]
    L.louvain_batch_graph_stats.restype = st
    L.louvain_batch_destroy.argtypes = [vp]
    L.louvain_batch_destroy.restype = None
    L.louvain_batch_init_graphs.argtypes = [i32, vp, vp, vp, vp, vp, u32, vp, ctypes.POINTER(vp)]
    L.louvain_batch_init_graphs.restype = st
    L.louvain_batch_last_error.argtypes = [vp]
    L.louvain_batch_last_error.restype = ctypes.c_char_p
    L.louvain_server_config_default.argtypes = [ctypes.POINTER(ServerConfig)]
    L.louvain_server_config_default.restype = None
    L.louvain_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(Params), ctypes.POINTER(vp)]
    L.louvain_server_create.restype = st
    L.louvain_server_submit.argtypes = [vp, i64, i64, vp, vp, vp, ctypes.POINTER(u64)]
    L.louvain_server_submit.restype = st
    L.louvain_server_submit_borrowed.argtypes = [vp, i64, i64, vp, vp, vp, ctypes.POINTER(u64)]
    L.louvain_server_submit_borrowed.restype = st
    L.louvain_server_poll.argtypes = [vp, u64, vp, ctypes.POINTER(JobResult), ctypes.POINTER(i32)]
    L.louvain_server_poll.restype = st
    L.louvain_server_release.argtypes = [vp, u64]
    L.louvain_server_release.restype = st
    L.louvain_server_wait_all.argtypes = [vp]
    L.louvain_server_wait_all.restype = st
    L.louvain_server_last_error.argtypes = [vp]
    L.louvain_server_last_error.restype = ctypes.c_char_p
    L.louvain_server_destroy.argtypes = [vp]
    L.louvain_server_destroy.restype = None
    _lib = L
    return L


def _check(status: int, handle=None):
    if status != OK:
        msg = lib().louvain_last_error(handle)
        raise LouvainError(status, msg.decode() if msg else "")


def params(**kw) -> Params:
    """louvain_params with the paper's defaults, overridden by keyword:
    vf, color, color_balance, singlet_rule, threshold_mode, color_first_phase_only, max_iter,
    max_phases, theta_color=(num, den), theta_final=(num, den), color_cutoff,
    color_seed."""
    p = Params()
    lib().louvain_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if k in ("theta_color", "theta_final"):
            setattr(p, k, Ratio(int(v[0]), int(v[1])))
        else:
            setattr(p, k, int(v))
    return p


def _stream_ptr(stream) -> Optional[int]:
    if stream == 0:
        return None  # the null stream
    if stream is None:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
        return None
    return getattr(stream, "cuda_stream", stream)


# ---- C-named functions --------------------------------------------------------
def louvain_init_csr(n, nnz, offsets, cols, weights=None, flags=VALIDATE, hip_stream=None) -> int:
    """Pointers are ints (device pointers with DEVICE_PTRS) or numpy arrays (host)."""
    def ptr(x):
        if x is None:
            return None
        if isinstance(x, np.ndarray):
            return x.ctypes.data
        return int(x)
    h = ctypes.c_void_p()
    _check(lib().louvain_init_csr(int(n), int(nnz), ptr(offsets), ptr(cols), ptr(weights), int(flags),
                                  _stream_ptr(hip_stream), ctypes.byref(h)))
    return h.value


def louvain_vf(h) -> int:
    out = ctypes.c_int64()
    _check(lib().louvain_vf(h, ctypes.byref(out)), h)
    return out.value


def louvain_vf_chain(h):
    """Chain-compressing vertex following: (vertices after, rounds that merged)."""
    out = ctypes.c_int64()
    rounds = ctypes.c_int64()
    _check(lib().louvain_vf_chain(h, ctypes.byref(out), ctypes.byref(rounds)), h)
    return out.value, rounds.value


def louvain_color(h, seed=DEFAULT_SEED) -> int:
    out = ctypes.c_int32()
    _check(lib().louvain_color(h, seed, ctypes.byref(out)), h)
    return out.value


def louvain_color_balance(h, seed=DEFAULT_SEED) -> int:
    out = ctypes.c_int64()
    _check(lib().louvain_color_balance(h, seed, ctypes.byref(out)), h)
    return out.value


def louvain_sweep(h, p: Params) -> IterStats:
    out = IterStats()
    _check(lib().louvain_sweep(h, ctypes.byref(p), ctypes.byref(out)), h)
    return out


def louvain_coarsen(h) -> int:
    out = ctypes.c_int64()
    _check(lib().louvain_coarsen(h, ctypes.byref(out)), h)
    return out.value


def louvain_run(h, p: Params, labels_ptr=None, labels_on_device=0) -> Result:
    out = Result()
    _check(lib().louvain_run(h, ctypes.byref(p), labels_ptr, int(labels_on_device), ctypes.byref(out)), h)
    return out


def louvain_run_noalloc(n, nnz, offsets, cols, weights, p: Params, labels_ptr=None, flags=0,
                        hip_stream=None) -> Result:
    """The allocation-free run: offsets, cols, weights (or None) and labels_ptr
    are device pointers (ints); nothing is allocated on the device."""
    out = Result()
    _check(lib().louvain_run_noalloc(int(n), int(nnz), offsets, cols, weights, int(flags), ctypes.byref(p),
                                     labels_ptr, _stream_ptr(hip_stream), ctypes.byref(out)))
    return out


def louvain_destroy(h):
    lib().louvain_destroy(h)


def louvain_last_error(h=None) -> str:
    m = lib().louvain_last_error(h)
    return m.decode() if m else ""


# ---- convenience wrapper ----------------------------------------------------------
@dataclass
class PhaseInfo:
    n: int
    nnz: int
    colored: bool
    num_colors: int
    iterations: int
    hit_max_iter: bool
    moves: List[int]
    N_iter: List[int]
    N_end: int
    pairs: List[int]
    entries: List[int]
    ms_color: float
    ms_sweep: float
    ms_coarsen: float
    undone: bool = False


@dataclass
class RunResult:
    labels: Optional[np.ndarray]
    K: int
    N: int
    D: int
    q: float
    n_vf: int
    N0: int
    sweep_entries: int
    ms_total: float
    ms_vf: float
    ms_color: float
    ms_sweep: float
    ms_coarsen: float
    phases: List[PhaseInfo] = field(default_factory=list)
    lookahead_entries: int = 0
    vf_rounds: int = 0


def _convert(res: Result, labels) -> RunResult:
    iters = [res.iter[t] for t in range(res.iterations)]
    phases = []
    for p in range(res.phases):
        ph = res.phase[p]
        its = iters[ph.first_iter:ph.first_iter + ph.iterations]
        phases.append(PhaseInfo(n=ph.n, nnz=ph.nnz, colored=bool(ph.colored), num_colors=ph.num_colors,
                                iterations=ph.iterations, hit_max_iter=bool(ph.hit_max_iter),
                                moves=[it.moves for it in its], N_iter=[it.q_num.value() for it in its],
                                N_end=ph.q_num.value(), pairs=[it.pairs for it in its],
                                entries=[it.entries for it in its], ms_color=ph.ms_color,
                                ms_sweep=ph.ms_sweep, ms_coarsen=ph.ms_coarsen, undone=bool(ph.loss_undone)))
    return RunResult(labels=labels, K=res.num_communities, N=res.q_num.value(), D=res.q_den.value(), q=res.q,
                     n_vf=res.n_vf, N0=res.q0_num.value(), sweep_entries=res.sweep_entries,
                     ms_total=res.ms_total, ms_vf=res.ms_vf, ms_color=res.ms_color, ms_sweep=res.ms_sweep,
                     ms_coarsen=res.ms_coarsen, phases=phases, lookahead_entries=res.lookahead_entries,
                     vf_rounds=res.vf_rounds)


class Graph:
    """One library handle.  Build from a host CSR (numpy) or from device
    tensors (torch)."""

    def __init__(self, handle: int):
        self.h = handle

    @classmethod
    def from_csr(cls, g, validate: bool = True, stream=None) -> "Graph":
        off = np.ascontiguousarray(g.offsets, dtype=np.int64)
        col = np.ascontiguousarray(g.cols, dtype=np.int32)
        w = None if g.weights is None else np.ascontiguousarray(g.weights, dtype=np.int32)
        return cls(louvain_init_csr(g.n, int(off[-1]), off, col, w, VALIDATE if validate else 0, stream))

    @classmethod
    def from_tensors(cls, offsets, cols, weights=None, validate: bool = False, stream=None) -> "Graph":
        n = offsets.numel() - 1
        nnz = cols.numel()
        flags = DEVICE_PTRS | (VALIDATE if validate else 0)
        return cls(louvain_init_csr(n, nnz, offsets.data_ptr(), cols.data_ptr(),
                                    None if weights is None else weights.data_ptr(), flags, stream))

    def close(self):
        if self.h:
            louvain_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # steps
    def vf_chain(self):
        return louvain_vf_chain(self.h)

    def vf(self) -> int:
        return louvain_vf(self.h)

    def balance(self, seed: int = DEFAULT_SEED) -> int:
        return louvain_color_balance(self.h, seed)

    def color(self, seed: int = DEFAULT_SEED) -> int:
        return louvain_color(self.h, seed)

    def sweep(self, p: Optional[Params] = None, **kw) -> dict:
        s = louvain_sweep(self.h, p or params(**kw))
        return {"moves": s.moves, "N": s.q_num.value(), "pairs": s.pairs, "entries": s.entries}

    def coarsen(self) -> int:
        return louvain_coarsen(self.h)

    def run(self, p: Optional[Params] = None, labels=None, **kw) -> RunResult:
        """labels: None (host copy returned), or a torch int32 device tensor of n_orig."""
        p = p or params(**kw)
        info = self.info()
        if labels is None:
            out = np.zeros(max(info["n_orig"], 1), dtype=np.int32)
            res = louvain_run(self.h, p, out.ctypes.data, 0)
            return _convert(res, out[:info["n_orig"]])
        res = louvain_run(self.h, p, labels.data_ptr(), 1)
        return _convert(res, None)

    # inspection
    def info(self) -> dict:
        out = np.zeros(8, dtype=np.int64)
        _check(lib().louvain_get_info(self.h, out.ctypes.data), self.h)
        return {"n": int(out[0]), "nnz": int(out[1]), "two_m": int(out[2]), "n_orig": int(out[3]),
                "num_colors": int(out[4]), "weight_kind": int(out[5]), "k_max": int(out[6]), "level": int(out[7])}

    def state(self) -> dict:
        n = self.info()["n"]
        comm = np.zeros(max(n, 1), np.int32)
        a = np.zeros(max(n, 1), np.int64)
        size = np.zeros(max(n, 1), np.int32)
        k = np.zeros(max(n, 1), np.int64)
        _check(lib().louvain_get_state(self.h, comm.ctypes.data, a.ctypes.data, size.ctypes.data, k.ctypes.data, 0),
               self.h)
        return {"comm": comm[:n], "a": a[:n], "size": size[:n], "k": k[:n]}

    def graph(self):
        info = self.info()
        n, nnz = info["n"], info["nnz"]
        off = np.zeros(n + 1, np.int64)
        col = np.zeros(max(nnz, 1), np.int32)
        w = np.zeros(max(nnz, 1), np.int64)
        _check(lib().louvain_get_graph(self.h, off.ctypes.data, col.ctypes.data, w.ctypes.data, 0), self.h)
        return off, col[:nnz], w[:nnz]

    def colors(self) -> np.ndarray:
        n = self.info()["n"]
        out = np.zeros(max(n, 1), np.int32)
        _check(lib().louvain_get_colors(self.h, out.ctypes.data, 0), self.h)
        return out[:n]

    def orig_map(self) -> np.ndarray:
        n0 = self.info()["n_orig"]
        out = np.zeros(max(n0, 1), np.int32)
        _check(lib().louvain_get_map(self.h, out.ctypes.data, 0), self.h)
        return out[:n0]

    def profile(self, enable: bool = True):
        _check(lib().louvain_profile(self.h, 1 if enable else 0), self.h)

    def profile_records(self) -> list:
        recs = []
        idx = 0
        while True:
            name = ctypes.c_char_p()
            launches = ctypes.c_int64()
            ms = ctypes.c_double()
            byts = ctypes.c_double()
            ent = ctypes.c_double()
            st = lib().louvain_profile_get(self.h, idx, ctypes.byref(name), ctypes.byref(launches), ctypes.byref(ms),
                                           ctypes.byref(byts), ctypes.byref(ent))
            if st != OK:
                break
            recs.append({"name": name.value.decode(), "launches": launches.value, "ms": ms.value,
                         "bytes": byts.value, "entries": ent.value})
            idx += 1
        return recs


# ---- batched form ---------------------------------------------------------------
def union_csr(graphs):
    """Packs graphs into one disjoint-union CSR: (graph_off, offsets, cols, weights)."""
    ns = [g.n for g in graphs]
    goff = np.zeros(len(graphs) + 1, dtype=np.int64)
    goff[1:] = np.cumsum(ns)
    weighted = any(g.weights is not None for g in graphs)
    offs, cols, ws = [np.zeros(1, dtype=np.int64)], [], []
    base_e = 0
    for gi, g in enumerate(graphs):
        offs.append(g.offsets[1:] + base_e)
        cols.append(g.cols.astype(np.int64) + goff[gi])
        if weighted:
            ws.append(np.ones(g.nnz, np.int32) if g.weights is None else g.weights)
        base_e += g.nnz
    off = np.concatenate(offs).astype(np.int64)
    col = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    w = np.concatenate(ws).astype(np.int32) if weighted and ws else None
    return goff, off, col, w


def louvain_batch_init(num_graphs, graph_off, nnz, offsets, cols, weights=None, flags=VALIDATE, hip_stream=None):
    def ptr(x):
        if x is None:
            return None
        if isinstance(x, np.ndarray):
            return x.ctypes.data
        return int(x)
    h = ctypes.c_void_p()
    goff = np.ascontiguousarray(graph_off, dtype=np.int64)
    st = lib().louvain_batch_init(int(num_graphs), goff.ctypes.data, int(nnz), ptr(offsets), ptr(cols), ptr(weights),
                                  int(flags), _stream_ptr(hip_stream), ctypes.byref(h))
    if st != OK:
        raise LouvainError(st, lib().louvain_batch_last_error(None).decode())
    return h.value


class Batch:
    """Many graphs run together by the batched kernels."""

    def __init__(self, graphs, validate: bool = True, stream=None):
        self.graphs = list(graphs)
        goff, off, col, w = union_csr(self.graphs)
        self.goff = goff
        self.h = louvain_batch_init(len(self.graphs), goff, int(off[-1]), off, col, w,
                                    VALIDATE if validate else 0, stream)

    @classmethod
    def from_graphs(cls, graphs, validate: bool = True, stream=None):
        """Separate host CSRs, packed on the device (louvain_batch_init_graphs)."""
        self = cls.__new__(cls)
        self.graphs = list(graphs)
        ng = len(self.graphs)
        keep = []  # contiguous arrays alive until the call returns

        def arr(x, dt):
            a = np.ascontiguousarray(x, dtype=dt)
            keep.append(a)
            return a.ctypes.data
        ns = np.array([g.n for g in self.graphs], dtype=np.int64)
        nnz = np.array([g.nnz for g in self.graphs], dtype=np.int64)
        P = ctypes.c_void_p * max(ng, 1)
        offs = P(*[arr(g.offsets, np.int64) for g in self.graphs])
        cols = P(*[arr(g.cols, np.int32) if g.nnz else None for g in self.graphs])
        weighted = any(g.weights is not None for g in self.graphs)
        ws = P(*[arr(g.weights, np.int32) if g.weights is not None else None for g in self.graphs]) if weighted else None
        self.goff = np.zeros(ng + 1, dtype=np.int64)
        self.goff[1:] = np.cumsum(ns)
        h = ctypes.c_void_p()
        st = lib().louvain_batch_init_graphs(ng, ns.ctypes.data, nnz.ctypes.data, offs, cols, ws,
                                             VALIDATE if validate else 0, _stream_ptr(stream), ctypes.byref(h))
        if st != OK:
            raise LouvainError(st, lib().louvain_batch_last_error(None).decode())
        self.h = h.value
        return self

    @classmethod
    def from_union(cls, graph_off, offsets, cols, weights=None, device=True, stream=None):
        """Device tensors (torch) of a union CSR already in HBM."""
        self = cls.__new__(cls)
        self.graphs = None
        self.goff = np.ascontiguousarray(graph_off, dtype=np.int64)
        self.h = louvain_batch_init(len(self.goff) - 1, self.goff, cols.numel(), offsets.data_ptr(),
                                    cols.data_ptr(), None if weights is None else weights.data_ptr(),
                                    DEVICE_PTRS, stream)
        return self

    def close(self):
        if getattr(self, "h", None):
            lib().louvain_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, p: Optional[Params] = None, labels=None, stats: bool = True, **kw):
        """Returns (list of per-graph RunResult, labels array of the union) ;
        labels may be a torch int32 device tensor (then results carry no labels)."""
        p = p or params(**kw)
        ng = len(self.goff) - 1
        res = (GraphResult * max(ng, 1))()
        n = int(self.goff[-1])
        host = labels is None
        out = np.zeros(max(n, 1), dtype=np.int32) if host else None
        st = lib().louvain_batch_run(self.h, ctypes.byref(p), out.ctypes.data if host else labels.data_ptr(),
                                     0 if host else 1, res)
        if st != OK:
            raise LouvainError(st, lib().louvain_batch_last_error(self.h).decode())
        results = []
        for gi in range(ng):
            r = res[gi]
            phases = []
            if stats:
                pp = ctypes.POINTER(PhaseStats)()
                ip = ctypes.POINTER(IterStats)()
                npn = ctypes.c_int64()
                nin = ctypes.c_int64()
                lib().louvain_batch_graph_stats(self.h, gi, ctypes.byref(pp), ctypes.byref(npn), ctypes.byref(ip),
                                                ctypes.byref(nin))
                iters = [ip[t] for t in range(nin.value)]
                for q in range(npn.value):
                    ph = pp[q]
                    its = iters[ph.first_iter:ph.first_iter + ph.iterations]
                    phases.append(PhaseInfo(n=ph.n, nnz=ph.nnz, colored=bool(ph.colored), num_colors=ph.num_colors,
                                            iterations=ph.iterations, hit_max_iter=bool(ph.hit_max_iter),
                                            moves=[it.moves for it in its], N_iter=[it.q_num.value() for it in its],
                                            N_end=ph.q_num.value(), pairs=[it.pairs for it in its],
                                            entries=[it.entries for it in its], ms_color=0.0, ms_sweep=0.0,
                                            ms_coarsen=0.0, undone=bool(ph.loss_undone)))
            lab = out[self.goff[gi]:self.goff[gi + 1]].copy() if host else None
            results.append(RunResult(labels=lab, K=r.num_communities, N=r.q_num.value(), D=r.q_den.value(), q=r.q,
                                     n_vf=r.n_vf, N0=r.q0_num.value(), sweep_entries=0, ms_total=0.0, ms_vf=0.0,
                                     ms_color=0.0, ms_sweep=0.0, ms_coarsen=0.0, phases=phases))
        return results


@dataclass
class JobInfo:
    """Outcome of one served job."""
    ticket: int
    status: int
    labels: Optional[np.ndarray]
    K: int
    N: int
    D: int
    q: float
    n_vf: int
    phases: int
    iterations: int
    t_submit: float
    t_admit: float
    t_done: float
    batch_id: int
    batch_graphs: int
    t_packed: float = 0.0
    t_ready: float = 0.0

    @property
    def latency(self) -> float:
        return self.t_done - self.t_submit


def louvain_server_config_default() -> ServerConfig:
    c = ServerConfig()
    lib().louvain_server_config_default(ctypes.byref(c))
    return c


class Server:
    """The served form: submit host CSRs, poll for results (continuous
    batching under an HBM budget, batches overlapping on their own streams)."""

    def __init__(self, p: Optional[Params] = None, hbm_budget_bytes: Optional[int] = None,
                 max_inflight_batches: Optional[int] = None, max_batch_graphs: Optional[int] = None,
                 max_batch_vertices: Optional[int] = None, solo_min_vertices: Optional[int] = None, **kw):
        cfg = louvain_server_config_default()
        if hbm_budget_bytes is not None:
            cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        if max_inflight_batches is not None:
            cfg.max_inflight_batches = int(max_inflight_batches)
        if max_batch_graphs is not None:
            cfg.max_batch_graphs = int(max_batch_graphs)
        if max_batch_vertices is not None:
            cfg.max_batch_vertices = int(max_batch_vertices)
        if solo_min_vertices is not None:
            cfg.solo_min_vertices = int(solo_min_vertices)
        self.p = p or params(**kw)
        h = ctypes.c_void_p()
        st = lib().louvain_server_create(ctypes.byref(cfg), ctypes.byref(self.p), ctypes.byref(h))
        if st != OK:
            raise LouvainError(st, "louvain_server_create rejected its arguments")
        self.h = h.value
        self.sizes = {}
        self.held = {}  # ticket -> arrays of a borrowed job, kept alive until it is done

    def submit(self, g, borrow: bool = False) -> int:
        """Queues a job; borrow=True skips the copy: the arrays are kept
        referenced here until the job is done."""
        off = np.ascontiguousarray(g.offsets, dtype=np.int64)
        col = np.ascontiguousarray(g.cols, dtype=np.int32)
        w = None if g.weights is None else np.ascontiguousarray(g.weights, dtype=np.int32)
        t = ctypes.c_uint64()
        fn = lib().louvain_server_submit_borrowed if borrow else lib().louvain_server_submit
        st = fn(self.h, int(g.n), int(col.size), off.ctypes.data, col.ctypes.data if col.size else None,
                None if w is None else w.ctypes.data, ctypes.byref(t))
        if st != OK:
            raise LouvainError(st, "louvain_server_submit rejected the graph")
        self.sizes[t.value] = int(g.n)
        if borrow:
            self.held[t.value] = (off, col, w)
        return t.value

    def poll(self, ticket: int, labels: bool = True) -> Optional[JobInfo]:
        n = self.sizes.get(ticket, 0)
        out = np.zeros(max(n, 1), dtype=np.int32) if labels else None
        r = JobResult()
        done = ctypes.c_int32()
        st = lib().louvain_server_poll(self.h, ticket, None if out is None else out.ctypes.data, ctypes.byref(r),
                                       ctypes.byref(done))
        if st != OK:
            raise LouvainError(st, "unknown ticket")
        if not done.value:
            return None
        self.held.pop(ticket, None)
        g = r.result
        return JobInfo(ticket=ticket, status=r.status, labels=None if out is None else out[:n],
                       K=g.num_communities, N=g.q_num.value(), D=g.q_den.value(), q=g.q, n_vf=g.n_vf,
                       phases=g.phases, iterations=g.iterations, t_submit=r.t_submit, t_admit=r.t_admit,
                       t_done=r.t_done, batch_id=r.batch_id, batch_graphs=r.batch_graphs, t_packed=r.t_packed,
                       t_ready=r.t_ready)

    def release(self, ticket: int):
        _ = lib().louvain_server_release(self.h, ticket)
        self.sizes.pop(ticket, None)

    def wait_all(self):
        st = lib().louvain_server_wait_all(self.h)
        self.held.clear()
        if st != OK:
            raise LouvainError(st, lib().louvain_server_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().louvain_server_destroy(self.h)
            self.h = None
            self.held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
