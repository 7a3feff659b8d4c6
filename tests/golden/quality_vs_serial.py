"""The quality study of the paper (Table 2's modularity columns, Table 3's
pair-counting agreement) on the synthetic workloads: the serial Louvain
method (Sec. 3) against the synchronous parallel heuristic with the paper's
settings.  The synchronous partition is the oracle's, which the HIP library
reproduces bit for bit (tests/golden).  Calls only oracle/.  Usage::

    python tests/golden/quality_vs_serial.py sbm_n1000:plain rmat_s20:full
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle import serial as S  # noqa: E402
from paper_1410_1237_amd import graphs as G  # noqa: E402

HEURISTICS = {"plain": {}, "full": {"vf": 1, "color": 1}}
# smaller members of the benchmark families, for the serial method's sake
EXTRA = {"chunglu_500k": lambda: G.chung_lu(500_000, 2.1, 12_500.0, 1.25e7, 6_250_000, wmax=100, seed=4)}


def main(targets):
    print("| workload | heuristics | K serial | Q serial | K parallel | Q parallel | SP | SE | OQ | Rand |")
    print("|---|---|---|---|---|---|---|---|---|---|")
    for t in targets:
        wl, heur = t.split(":")
        g = EXTRA[wl]() if wl in EXTRA else G.WORKLOADS[wl]()
        t0 = time.time()
        s = S.serial_louvain(g)
        t1 = time.time()
        p = oracle.default().run(g, oracle.Params(**HEURISTICS[heur]))
        m = S.agreement(s.labels, p.labels)
        print(f"| {wl} | {heur} | {s.K} | {s.q:.6f} | {p.K} | {p.q:.6f} | {100 * m['SP']:.2f}% | "
              f"{100 * m['SE']:.2f}% | {100 * m['OQ']:.2f}% | {100 * m['Rand']:.2f}% |", flush=True)
        print(f"<!-- serial {t1 - t0:.1f} s on one core -->", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["sbm_n1000:plain", "rmat_s20:full"])
