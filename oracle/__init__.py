"""ORACLE -- test infrastructure only.

ctypes wrapper around ``liboracle.so`` (built from ``oracle.cpp`` with g++):
a plain serial CPU implementation of the synchronous parallel Louvain
heuristic with exact integer arithmetic.  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark may import this package; the product
path (``paper_1410_1237_amd``) never does.

Modularity is returned as the exact pair (N, D) with Q = N / D,
N = 2m * (internal weight) - sum_C a_C^2 and D = (2m)^2 (Eq. 3 times (2m)^2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

DEFAULT_SEED = 0x4C4F5556


def build(src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle with g++ (plain host code)."""
    cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", out, src]
    subprocess.run(cmd, check=True)
    return out


def _i128(lo: int, hi: int) -> int:
    return (int(hi) << 64) | (int(lo) & ((1 << 64) - 1))


@dataclass
class Params:
    """Run parameters (defaults: the paper's baseline = minimum-label sweep,
    singlet rule on, relative threshold 1e-6, no VF, no coloring).  vf: 0
    none, 1 single-degree vertex following, 2 chain-compressing."""
    vf: int = 0
    color: int = 0
    singlet_rule: int = 1
    threshold_mode: int = 0
    color_first_phase_only: int = 0
    theta_color: tuple = (1, 100)
    theta_final: tuple = (1, 1000000)
    color_cutoff: int = 100000
    max_iter: int = 1000
    max_phases: int = 100
    color_seed: int = DEFAULT_SEED
    color_balance: int = 0

    def flat(self) -> np.ndarray:
        return np.array([self.vf, self.color, self.singlet_rule, self.threshold_mode,
                         self.color_first_phase_only, self.theta_color[0], self.theta_color[1],
                         self.theta_final[0], self.theta_final[1], self.color_cutoff,
                         self.max_iter, self.max_phases, self.color_seed, self.color_balance],
                        dtype=np.int64)


@dataclass
class Phase:
    n: int
    nnz: int
    colored: bool
    ncolors: int
    iterations: int
    hit_max_iter: bool
    moves: List[int]
    N_iter: List[int]
    N_end: int
    undone: bool = False


@dataclass
class Result:
    labels: np.ndarray
    K: int
    N: int
    D: int
    q: float
    n_vf: int
    N0: int
    phases: List[Phase] = field(default_factory=list)
    phase_labels: List[np.ndarray] = field(default_factory=list)
    vf_rounds: int = 0


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class Oracle:
    def __init__(self, lib: str = LIB):
        if not os.path.exists(lib):
            build(out=lib)
        L = ctypes.CDLL(lib)
        vp, i64, i32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
        L.oracle_validate.argtypes = [i64, vp, vp, vp]
        L.oracle_validate.restype = ctypes.c_int
        L.oracle_degrees.argtypes = [i64, vp, vp, vp, vp, vp]
        L.oracle_modularity.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp]
        L.oracle_mix64.argtypes = [u64]
        L.oracle_mix64.restype = u64
        L.oracle_ratio_to_double.argtypes = [i64, i64, i64, i64]
        L.oracle_ratio_to_double.restype = ctypes.c_double
        L.oracle_state_new.argtypes = [i64, vp, vp, vp]
        L.oracle_state_new.restype = vp
        L.oracle_state_free.argtypes = [vp]
        L.oracle_state_info.argtypes = [vp, vp]
        L.oracle_state_vf.argtypes = [vp]
        L.oracle_state_vf_chain.argtypes = [vp]
        L.oracle_state_vf_chain.restype = i64
        L.oracle_state_color.argtypes = [vp, u64]
        L.oracle_state_color.restype = i32
        L.oracle_state_uncolor.argtypes = [vp]
        L.oracle_state_balance.argtypes = [vp, u64]
        L.oracle_state_balance.restype = i64
        L.oracle_state_iterate.argtypes = [vp, i32, vp]
        L.oracle_state_iterate.restype = i64
        L.oracle_state_coarsen.argtypes = [vp]
        L.oracle_state_coarsen.restype = i64
        L.oracle_state_get.argtypes = [vp, i32, vp]
        L.oracle_state_set_comm.argtypes = [vp, vp]
        L.oracle_state_gain.argtypes = [vp, i64, i32, vp, vp]
        L.oracle_state_decide.argtypes = [vp, i64, i32]
        L.oracle_state_decide.restype = i32
        L.oracle_state_decide_range.argtypes = [vp, i64, i64, i32, vp]
        L.oracle_state_decide_range.restype = i64
        L.oracle_run.argtypes = [i64, vp, vp, vp, vp]
        L.oracle_run.restype = vp
        L.oracle_result_free.argtypes = [vp]
        L.oracle_result_scalars.argtypes = [vp, vp, vp]
        L.oracle_result_labels.argtypes = [vp, vp]
        L.oracle_result_phase_labels.argtypes = [vp, i64, vp]
        L.oracle_result_phase.argtypes = [vp, i64, vp]
        L.oracle_result_iter.argtypes = [vp, i64, vp]
        self.L = L

    # -- plain functions -------------------------------------------------
    @staticmethod
    def _arrays(g):
        off = np.ascontiguousarray(g.offsets, dtype=np.int64)
        col = np.ascontiguousarray(g.cols, dtype=np.int32)
        w = None if g.weights is None else np.ascontiguousarray(g.weights, dtype=np.int32)
        return off, col, w

    def validate(self, g) -> int:
        off, col, w = self._arrays(g)
        return int(self.L.oracle_validate(g.n, _ptr(off), _ptr(col), _ptr(w)))

    def degrees(self, g):
        off, col, w = self._arrays(g)
        k = np.zeros(g.n, dtype=np.int64)
        tm = np.zeros(1, dtype=np.int64)
        self.L.oracle_degrees(g.n, _ptr(off), _ptr(col), _ptr(w), _ptr(k), _ptr(tm))
        return k, int(tm[0])

    def modularity(self, g, labels, w64=None):
        """Exact (N, D) of a partition; g may carry int64 weights via w64."""
        off, col, w = self._arrays(g)
        if w64 is not None:
            w = None
            w64 = np.ascontiguousarray(w64, dtype=np.int64)
        lab = np.ascontiguousarray(labels, dtype=np.int32)
        N = np.zeros(2, dtype=np.int64)
        D = np.zeros(2, dtype=np.int64)
        self.L.oracle_modularity(g.n, _ptr(off), _ptr(col), _ptr(w), _ptr(w64), _ptr(lab),
                                 _ptr(N), _ptr(D))
        return _i128(N[0], N[1]), _i128(D[0], D[1])

    def mix64(self, z: int) -> int:
        return int(self.L.oracle_mix64(z & ((1 << 64) - 1)))

    def ratio_to_double(self, N: int, D: int) -> float:
        m = (1 << 64) - 1

        def split(x):
            lo = x & m
            hi = x >> 64
            lo = lo - (1 << 64) if lo >= (1 << 63) else lo
            return lo, hi
        nl, nh = split(N)
        dl, dh = split(D)
        return float(self.L.oracle_ratio_to_double(nl, nh, dl, dh))

    # -- step-wise state -------------------------------------------------
    def state(self, g) -> "State":
        return State(self, g)

    # -- full run --------------------------------------------------------
    def run(self, g, params: Optional[Params] = None, phase_labels: bool = False) -> Result:
        params = params or Params()
        off, col, w = self._arrays(g)
        pf = params.flat()
        h = self.L.oracle_run(g.n, _ptr(off), _ptr(col), _ptr(w), _ptr(pf))
        try:
            sc = np.zeros(12, dtype=np.int64)
            q = ctypes.c_double()
            self.L.oracle_result_scalars(h, _ptr(sc), ctypes.byref(q))
            labels = np.zeros(max(g.n, 1), dtype=np.int32)
            self.L.oracle_result_labels(h, _ptr(labels))
            iters = []
            for t in range(int(sc[4])):
                it = np.zeros(3, dtype=np.int64)
                self.L.oracle_result_iter(h, t, _ptr(it))
                iters.append((int(it[0]), _i128(it[1], it[2])))
            phases, plabels = [], []
            for p in range(int(sc[3])):
                ph = np.zeros(10, dtype=np.int64)
                self.L.oracle_result_phase(h, p, _ptr(ph))
                f, nit = int(ph[6]), int(ph[4])
                phases.append(Phase(n=int(ph[0]), nnz=int(ph[1]), colored=bool(ph[2]),
                                    ncolors=int(ph[3]), iterations=nit, hit_max_iter=bool(ph[5]),
                                    moves=[m for m, _ in iters[f:f + nit]],
                                    N_iter=[N for _, N in iters[f:f + nit]],
                                    N_end=_i128(ph[7], ph[8]), undone=bool(ph[9])))
                if phase_labels:
                    pl = np.zeros(max(g.n, 1), dtype=np.int32)
                    self.L.oracle_result_phase_labels(h, p, _ptr(pl))
                    plabels.append(pl[:g.n])
            return Result(labels=labels[:g.n], K=int(sc[1]), N=_i128(sc[5], sc[6]),
                          D=_i128(sc[7], sc[8]), q=q.value, n_vf=int(sc[2]), N0=_i128(sc[9], sc[10]),
                          phases=phases, phase_labels=plabels, vf_rounds=int(sc[11]))
        finally:
            self.L.oracle_result_free(h)


class State:
    """Step-wise oracle state on one graph: singletons at creation; vf(),
    color(), iterate(), coarsen() mirror the library's step calls."""

    def __init__(self, O: Oracle, g):
        self.O = O
        off, col, w = O._arrays(g)
        self.h = O.L.oracle_state_new(g.n, _ptr(off), _ptr(col), _ptr(w))

    def __del__(self):
        try:
            self.O.L.oracle_state_free(self.h)
        except Exception:
            pass

    def info(self):
        out = np.zeros(5, dtype=np.int64)
        self.O.L.oracle_state_info(self.h, _ptr(out))
        return {"n": int(out[0]), "nnz": int(out[1]), "two_m": int(out[2]),
                "ncolors": int(out[3]), "n_orig": int(out[4])}

    def vf(self):
        self.O.L.oracle_state_vf(self.h)

    def vf_chain(self) -> int:
        """Chain-compressing vertex following; returns the rounds that merged."""
        return int(self.O.L.oracle_state_vf_chain(self.h))

    def color(self, seed: int = DEFAULT_SEED) -> int:
        return int(self.O.L.oracle_state_color(self.h, seed))

    def balance(self, seed: int = DEFAULT_SEED) -> int:
        """Balanced colouring of the current colouring; returns the vertices moved."""
        return int(self.O.L.oracle_state_balance(self.h, seed))

    def uncolor(self):
        self.O.L.oracle_state_uncolor(self.h)

    def iterate(self, singlet_rule: int = 1):
        N = np.zeros(2, dtype=np.int64)
        moves = int(self.O.L.oracle_state_iterate(self.h, singlet_rule, _ptr(N)))
        return moves, _i128(N[0], N[1])

    def coarsen(self) -> int:
        return int(self.O.L.oracle_state_coarsen(self.h))

    def get(self, which: str) -> np.ndarray:
        info = self.info()
        n, nnz = info["n"], info["nnz"]
        spec = {"comm": (0, np.int32, n), "a": (1, np.int64, n), "size": (2, np.int32, n),
                "k": (3, np.int64, n), "color": (4, np.int32, n if info["ncolors"] else 0),
                "offsets": (5, np.int64, n + 1), "cols": (6, np.int32, nnz),
                "weights": (7, np.int64, nnz), "orig_map": (8, np.int32, info["n_orig"])}[which]
        out = np.zeros(max(spec[2], 1), dtype=spec[1])
        self.O.L.oracle_state_get(self.h, spec[0], _ptr(out))
        return out[:spec[2]]

    def set_comm(self, comm):
        c = np.ascontiguousarray(comm, dtype=np.int32)
        self.O.L.oracle_state_set_comm(self.h, _ptr(c))

    def gain(self, i: int, c: int):
        G = np.zeros(2, dtype=np.int64)
        S = np.zeros(2, dtype=np.int64)
        self.O.L.oracle_state_gain(self.h, i, c, _ptr(G), _ptr(S))
        return _i128(G[0], G[1]), _i128(S[0], S[1])

    def decide(self, i: int, singlet_rule: int = 1) -> int:
        return int(self.O.L.oracle_state_decide(self.h, i, singlet_rule))

    def decide_range(self, lo: int, hi: int, singlet_rule: int = 1):
        """Decisions of vertices [lo, hi) against the current state; returns
        (decisions, CSR entries of those rows)."""
        out = np.zeros(max(hi - lo, 1), dtype=np.int32)
        ent = int(self.O.L.oracle_state_decide_range(self.h, lo, hi, singlet_rule, _ptr(out)))
        return out[:hi - lo], ent


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default
