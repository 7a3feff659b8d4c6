"""SERIAL BASELINE -- test and baseline infrastructure only.

ctypes wrapper around ``libserial.so`` (built from ``serial_louvain.cpp``):
the sequential Louvain method of Sec. 3 (in-order visits, each move applied
at once), the comparison system of the paper's quality study, and the
pair-counting agreement measures of that study (Sec. 6.2, Table 3): with S
the serial partition and P the parallel one, a vertex pair is a true
positive if it shares a community in both, a false positive if only in P, a
false negative if only in S and a true negative otherwise; then
SP = TP/(TP+FP), SE = TP/(TP+FN), OQ = TP/(TP+FP+FN) and
Rand = (TP+TN)/(all pairs).  The counts come from the contingency table of
the two partitions (pairs inside each non-empty cell, row and column), in
O(n log n) instead of the Theta(n^2) pair enumeration.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "serial_louvain.cpp")
LIB = os.path.join(HERE, "libserial.so")


def build(src: str = SRC, out: str = LIB) -> str:
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", out, src], check=True)
    return out


@dataclass
class SerialResult:
    labels: np.ndarray
    K: int
    N: int
    D: int
    phases: int
    iterations: int

    @property
    def q(self) -> float:
        from fractions import Fraction
        return float(Fraction(self.N, self.D))


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.serial_louvain_run.argtypes = [i64, vp, vp, vp, i64, i64, i32, i32, vp, vp]
        L.serial_louvain_run.restype = None
        _lib = L
    return _lib


def _i128(lo, hi) -> int:
    return (int(hi) << 64) | (int(lo) & ((1 << 64) - 1))


def serial_louvain(g, theta=(1, 1000000), max_iter: int = 1000, max_phases: int = 100) -> SerialResult:
    """The sequential Louvain method on graph g (a CSR with offsets, cols,
    weights or None), relative threshold theta = (num, den)."""
    off = np.ascontiguousarray(g.offsets, dtype=np.int64)
    col = np.ascontiguousarray(g.cols, dtype=np.int32)
    w = None if g.weights is None else np.ascontiguousarray(g.weights, dtype=np.int32)
    lab = np.zeros(max(g.n, 1), dtype=np.int32)
    out = np.zeros(7, dtype=np.int64)
    _load().serial_louvain_run(g.n, off.ctypes.data, col.ctypes.data, None if w is None else w.ctypes.data,
                               int(theta[0]), int(theta[1]), int(max_iter), int(max_phases), lab.ctypes.data,
                               out.ctypes.data)
    return SerialResult(labels=lab[:g.n], K=int(out[0]), phases=int(out[1]), iterations=int(out[2]),
                        N=_i128(out[3], out[4]), D=_i128(out[5], out[6]))


def _pairs(x: np.ndarray) -> int:
    x = x.astype(np.int64)
    return int((x * (x - 1) // 2).sum())


def pair_counts(S, P) -> dict:
    """TP, FP, FN, TN over all vertex pairs of partitions S (reference) and P."""
    S = np.asarray(S, dtype=np.int64)
    P = np.asarray(P, dtype=np.int64)
    assert S.shape == P.shape
    n = S.size
    _, s_sizes = np.unique(S, return_counts=True)
    _, p_sizes = np.unique(P, return_counts=True)
    _, cell = np.unique(np.stack([S, P], axis=1), axis=0, return_counts=True) if n else (None, np.zeros(0))
    tp = _pairs(cell)
    same_p, same_s = _pairs(p_sizes), _pairs(s_sizes)
    fp, fn = same_p - tp, same_s - tp
    tn = n * (n - 1) // 2 - tp - fp - fn
    return {"TP": tp, "FP": fp, "FN": fn, "TN": tn}


def agreement(S, P) -> dict:
    """SP, SE, OQ and Rand index of P against the reference S (Table 3's
    measures), as fractions; a measure whose denominator is 0 is reported as 1
    (no pair to disagree on)."""
    c = pair_counts(S, P)
    tp, fp, fn, tn = c["TP"], c["FP"], c["FN"], c["TN"]

    def ratio(a, b):
        return 1.0 if b == 0 else a / b
    return {"SP": ratio(tp, tp + fp), "SE": ratio(tp, tp + fn), "OQ": ratio(tp, tp + fp + fn),
            "Rand": ratio(tp + tn, tp + fp + fn + tn), **c}
