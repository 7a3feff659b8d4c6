"""Writes the stored expected results of the full-size workloads.

Every value here comes from the serial oracle (``oracle/``) run on the seeded
synthetic graphs of ``paper_1410_1237_amd.graphs``; nothing is taken from the
HIP library.  Usage::

    python tests/golden/make_golden.py rmat_s20:full rmat_s20:plain ...

Each target writes ``<workload>_<heuristics>.json`` beside this script with
the number of communities, the exact modularity pair (N, D), the
per-phase shape (vertices, entries, colouring, colours, iterations, moves and
exact per-iteration modularity numerators) and the SHA-256 of the final
labels (int32, little endian).
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1410_1237_amd import graphs as G  # noqa: E402

HEURISTICS = {
    # minimum-label synchronous sweeps, singlet rule, relative threshold 1e-6
    "plain": {},
    # vertex following + colouring (cutoff 100,000, 1e-2) + final 1e-6
    "full": {"vf": 1, "color": 1},
}


def labels_sha(labels) -> str:
    return hashlib.sha256(np.ascontiguousarray(labels, dtype="<i4").tobytes()).hexdigest()


def golden(workload: str, heur: str) -> dict:
    g = G.WORKLOADS[workload]()
    t = time.time()
    r = oracle.default().run(g, oracle.Params(**HEURISTICS[heur]))
    secs = time.time() - t
    return {
        "workload": workload, "heuristics": heur, "n": g.n, "nnz": g.nnz,
        "K": r.K, "N": str(r.N), "D": str(r.D), "q": r.q, "n_vf": r.n_vf, "N0": str(r.N0),
        "labels_sha256": labels_sha(r.labels),
        "phases": [{"n": p.n, "nnz": p.nnz, "colored": p.colored, "ncolors": p.ncolors,
                    "iterations": p.iterations, "moves": p.moves, "N_iter": [str(x) for x in p.N_iter],
                    "N_end": str(p.N_end), "undone": p.undone} for p in r.phases],
        "oracle_seconds": round(secs, 1),
    }


def main(targets):
    for t in targets:
        wl, heur = t.split(":")
        out = golden(wl, heur)
        path = os.path.join(HERE, f"{wl}_{heur}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(f"wrote {path}: K={out['K']} q={out['q']:.6f} ({out['oracle_seconds']} s)", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["sbm_n1000:plain", "rmat_s20:full", "rmat_s20:plain"])
