"""Writes the stored expected results of the full-size workloads.

Every value here comes from the serial oracle (``oracle/``) run on the seeded
synthetic graphs of ``paper_1410_1237_amd.graphs``; nothing is taken from the
HIP library.  Usage::

    python tests/golden/make_golden.py rmat_s20:full rmat_s20:plain ...
    python tests/golden/make_golden.py batch_sbm:4096 served:128

Each target writes ``<workload>_<heuristics>.json`` beside this script with
the number of communities, the exact modularity pair (N, D), the
per-phase shape (vertices, entries, colouring, colours, iterations, moves and
exact per-iteration modularity numerators) and the SHA-256 of the final
labels (int32, little endian).  A mix target (``batch_sbm:<count>``,
``served:<count>``) writes one compact record per graph of the batched or
served mix instead.
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


MIXES = {
    # the batched mix: planted SBMs of uneven sizes (batch_sbm(i))
    "batch_sbm": G.batch_sbm,
    # the served mix: SBM and R-MAT jobs from 1e3 to 2e6 vertices (served_job(i))
    "served": G.served_job,
}


def golden_mix(mix: str, count: int, threads: int) -> dict:
    """Oracle results of graphs 0..count-1 of a mix, plain heuristics, one
    compact record per graph: [i, n, nnz, K, N, D, phases, iterations,
    first 16 hex digits of the labels' SHA-256].  The graphs are independent:
    they run on a thread pool (the oracle and the generator release the GIL)."""
    import concurrent.futures as cf
    O = oracle.default()

    def one(i):
        g = MIXES[mix](i)
        r = O.run(g, oracle.Params())
        return [i, g.n, g.nnz, r.K, str(r.N), str(r.D), len(r.phases), sum(p.iterations for p in r.phases),
                labels_sha(r.labels)[:16]]
    t = time.time()
    # largest first, so that the pool's tail is short
    order = sorted(range(count), key=lambda i: -MIXES[mix + "_n"](i)) if mix + "_n" in MIXES else range(count)
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        recs = sorted(ex.map(one, order), key=lambda r: r[0])
    return {"mix": mix, "count": count, "heuristics": "plain",
            "fields": ["i", "n", "nnz", "K", "N", "D", "phases", "iterations", "labels_sha256_16"],
            "graphs": recs, "oracle_seconds": round(time.time() - t, 1), "threads": threads}


MIXES["batch_sbm_n"] = lambda i: G.batch_sbm_params(i)["n"]
MIXES["served_n"] = lambda i: G.served_job_params(i)["n"]


def main(targets):
    for t in targets:
        wl, heur = t.split(":")
        if wl in ("batch_sbm", "served"):
            count = int(heur)
            threads = int(os.environ.get("GOLDEN_THREADS", "8"))
            out = golden_mix(wl, count, threads)
            path = os.path.join(HERE, f"{wl}_x{count}_plain.json")
            with open(path, "w") as f:
                f.write("{\n")
                items = [(k, v) for k, v in out.items() if k != "graphs"]
                for k, v in items:
                    f.write(f" {json.dumps(k)}: {json.dumps(v)},\n")
                f.write(' "graphs": [\n')
                f.write(",\n".join("  " + json.dumps(r) for r in out["graphs"]))
                f.write("\n ]\n}\n")
            print(f"wrote {path}: {count} graphs ({out['oracle_seconds']} s)", flush=True)
            continue
        out = golden(wl, heur)
        path = os.path.join(HERE, f"{wl}_{heur}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(f"wrote {path}: K={out['K']} q={out['q']:.6f} ({out['oracle_seconds']} s)", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["sbm_n1000:plain", "rmat_s20:full", "rmat_s20:plain"])
