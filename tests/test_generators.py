"""Input generators: Philox known answers, CSR well-formedness, and outputs
independent of the host thread count."""
import hashlib
import os
import subprocess
import sys

import numpy as np

from paper_1410_1237_amd import graphs as G


def test_philox_known_answers():
    # Random123 known-answer vectors for Philox4x32-10
    assert G.philox4x32_10((0, 0, 0, 0), (0, 0)) == (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)
    f = 0xFFFFFFFF
    assert G.philox4x32_10((f, f, f, f), (f, f)) == (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)


def _well_formed(g):
    off, col = g.offsets, g.cols
    assert off[0] == 0 and off[-1] == len(col) and np.all(np.diff(off) >= 0)
    rows = np.repeat(np.arange(g.n), np.diff(off))
    assert np.all(col >= 0) and np.all(col < g.n)
    assert not np.any(rows == col)                      # no self-loops generated
    key = rows.astype(np.int64) * g.n + col
    assert np.all(np.diff(key) > 0)                      # sorted, unique per row
    mirror = col.astype(np.int64) * g.n + rows
    order = np.argsort(mirror)
    assert np.array_equal(mirror[order], key)           # symmetric
    if g.weights is not None:
        assert np.array_equal(g.weights[order], g.weights)
        assert g.weights.min() >= 1


def test_sbm_1000_shape():
    g = G.sbm_1000()
    _well_formed(g)
    assert g.n == 1000 and 11000 < g.nnz < 12400           # E[nnz] = 11,700
    blk = np.repeat(np.arange(g.n), np.diff(g.offsets)) // 100
    inside = (blk == g.cols // 100).mean()
    assert 0.80 < inside < 0.90                             # E = 9,900 / 11,700


def test_weighted_families():
    for g in (G.batch_sbm(3), G.rmat(12, 8, wmax=100, seed=9),
              G.chung_lu(20000, 2.1, 2000.0, 3.0e5, 150000, wmax=100, seed=4), G.served_job(5)):
        _well_formed(g)
    g = G.chung_lu(20000, 2.1, 2000.0, 3.0e5, 150000, wmax=100, seed=4)
    assert g.nnz == 300000
    assert 1 <= g.weights.min() and g.weights.max() <= 100


def _digest_cmd(threads):
    code = ("import hashlib;from paper_1410_1237_amd import graphs as G;"
            "g=G.rmat(14,16,seed=3);h=G.chung_lu(30000,2.1,3000.0,4e5,200000,100,4);"
            "print(hashlib.sha256(g.offsets.tobytes()+g.cols.tobytes()+h.cols.tobytes()+h.weights.tobytes()).hexdigest())")
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    return subprocess.run([sys.executable, "-c", code], env=env, cwd=root, check=True,
                          capture_output=True, text=True).stdout.strip()


def test_thread_count_independent():
    assert _digest_cmd(1) == _digest_cmd(5)
