"""The serial Louvain baseline (Sec. 3: in-order visits, each move applied at
once) and the pair-counting agreement measures of Table 3, against facts
outside their code: brute-force enumeration of vertex pairs, hand-worked
cases, closed forms of clique graphs, the modularity-matrix form of Q and
the brute-force optimum of tiny graphs."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import pins
import small_graphs as SG
from oracle import serial as S


def brute_pairs(a, b):
    tp = fp = fn = tn = 0
    for u, v in itertools.combinations(range(len(a)), 2):
        sa, sb = a[u] == a[v], b[u] == b[v]
        tp += sa and sb
        fp += sb and not sa
        fn += sa and not sb
        tn += not sa and not sb
    return {"TP": tp, "FP": fp, "FN": fn, "TN": tn}


def test_pair_counts_equal_pair_enumeration():
    rng = np.random.default_rng(3)
    for _ in range(60):
        n = int(rng.integers(0, 40))
        a = rng.integers(0, max(1, int(rng.integers(1, 8))), size=n)
        b = rng.integers(0, max(1, int(rng.integers(1, 8))), size=n) if rng.random() < 0.7 else a.copy()
        assert S.pair_counts(a, b) == brute_pairs(a.tolist(), b.tolist())


def test_agreement_measures_by_hand():
    # S = {0,1,2},{3,4}; P = {0,1},{2,3,4}: same in S: 01 02 12 34; same in P:
    # 01 23 24 34; TP = {01, 34}, FP = {23, 24}, FN = {02, 12}, TN = 4 of 10
    m = S.agreement([0, 0, 0, 1, 1], [0, 0, 1, 1, 1])
    assert (m["TP"], m["FP"], m["FN"], m["TN"]) == (2, 2, 2, 4)
    assert (m["SP"], m["SE"], m["OQ"], m["Rand"]) == (0.5, 0.5, 2 / 6, 0.6)
    # identical partitions score 1 everywhere (the paper's remark under Table 3)
    lab = np.array([3, 3, 1, 0, 1, 3])
    m = S.agreement(lab, lab.copy())
    assert (m["SP"], m["SE"], m["OQ"], m["Rand"]) == (1.0, 1.0, 1.0, 1.0)
    # relabelling does not matter, only the grouping
    m = S.agreement(lab, 10 - lab)
    assert m["OQ"] == 1.0 and m["FP"] == 0 and m["FN"] == 0


def test_serial_hand_cases():
    # one edge: vertex 0 joins 1 at once (G = 2m*1 - 1*1 = 1 > 0); vertex 1
    # then sees itself with 0 and stays: one community, Q = 0
    r = S.serial_louvain(SG.from_edges(2, [(0, 1)]))
    assert r.labels.tolist() == [0, 0] and (r.N, r.D) == (0, 4)
    # path 0-1-2 (2m = 4): 0 joins 1 (gain 2); 1 now has G_stay = 4*1 - 2*(3-2)
    # = 2 against G(C(2)) = 4 - 2*1 = 2, not better, stays; 2 joins 1
    # (G = 4 - 1*3 = 1 > 0): all together, Q = 0
    r = S.serial_louvain(SG.from_edges(3, [(0, 1), (1, 2)]))
    assert r.labels.tolist() == [0, 0, 0] and r.N == 0
    # the synchronous rule on the same path moves 0 and 2 towards 1 and 1
    # towards 0 in the same step; the serial one never loses (see below)


def test_serial_cliques_and_rings():
    rng = np.random.default_rng(5)
    for r_, s_ in [(2, 3), (3, 4), (5, 5)]:
        perm = rng.permutation(r_ * s_)
        g = SG.cliques(r_, s_, perm)
        res = S.serial_louvain(g)
        assert res.K == r_ and Fraction(res.N, res.D) == 1 - Fraction(1, r_)
    for r_, s_ in [(3, 3), (4, 5), (6, 5)]:
        res = S.serial_louvain(SG.ring_of_cliques(r_, s_))
        assert res.K == r_
        assert Fraction(res.N, res.D) == 1 - Fraction(2, s_ * (s_ - 1) + 2) - Fraction(1, r_)


def test_serial_q_is_the_partitions_q_and_bounded_by_optimum():
    rng = np.random.default_rng(11)
    for t in range(10):
        n = int(rng.integers(4, 10))
        g = SG.random_graph(rng, n, p=0.4, self_loops=0.2 if t % 2 else 0.0, wmax=5)
        res = S.serial_louvain(g)
        if res.D == 1:
            continue
        assert pins.n_modmatrix(g, res.labels) == (res.N, res.D)
        best, D = pins.best_partition_N(g)
        assert res.N <= best
        # never below the singletons: every serial move raises Q
        k = pins.dense(g).sum(axis=1)
        assert res.N >= int(k.sum()) * int(np.trace(pins.dense(g))) - int((k * k).sum())


@pytest.mark.parametrize("seed", [1, 2])
def test_serial_against_sbm_planted_partition(seed):
    """Plausibility on the 1,000-vertex SBM: both methods find the planted
    blocks almost exactly."""
    from paper_1410_1237_amd import graphs as GG
    import oracle
    g = GG.sbm_1000() if seed == 1 else GG.sbm(600, 6, 0.12, 0.003, seed=seed)
    ser = S.serial_louvain(g)
    syn = oracle.default().run(g)
    m = S.agreement(ser.labels, syn.labels)
    assert m["Rand"] > 0.99 and m["OQ"] > 0.9
