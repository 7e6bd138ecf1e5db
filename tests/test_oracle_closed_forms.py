"""Closed forms and textbook reductions that pin the FP64 oracle.

Each expected value below is derived by hand from the model definition (pair
HMM with virtual begin/end match states and no X-Y adjacency; partition
function over the same alignment set with affine gap scores at temperature T)
or computed by an independent textbook algorithm written here (an affine-gap
max-plus alignment with co-optimal counting; combinatorial alignment counts).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf
from paper_1512_07437_amd import workload as W


def _odds(p):
    q = p.joint.sum(1)
    return p.joint / np.outer(q, q)


def _g(L, p):
    """Weight of one HMM gap run of length L summed over its class label."""
    return sum(d * e ** (L - 1) * (1 - e) for d, e in zip(p.gap_open, p.gap_extend))


def test_1x1(params):
    x, y = W.encode("W"), W.encode("C")
    r = oracle.pair(x, y, params)
    assert abs(r["post"][0, 0] - 1.0) < 1e-14
    tau = 1 - 2 * sum(params.gap_open)
    e = _odds(params)[x[0], y[0]]
    # the only alignment: begin -> M -> end, weight tau^2 e
    assert abs(r["logz_h"] - math.log(tau * tau * e)) < 1e-13
    assert abs(r["logz_p"] - params.score[x[0], y[0]] / params.temperature) < 1e-13
    assert abs(r["ea"] - 1.0) < 1e-14


@pytest.mark.parametrize("xs,ys", [("AW", "W"), ("KL", "R"), ("CC", "C")])
def test_2x1(params, xs, ys):
    # two alignments: M(1,1) X(2) and X(1) M(2,1); each has one gap run of
    # length 1 and one M->M transition, so the gap terms cancel.
    x, y = W.encode(xs), W.encode(ys)
    r = oracle.pair(x, y, params)
    e = _odds(params)
    e1, e2 = e[x[0], y[0]], e[x[1], y[0]]
    assert abs(r["post_h"][0, 0] - e1 / (e1 + e2)) < 1e-14
    assert abs(r["post_h"][1, 0] - e2 / (e1 + e2)) < 1e-14
    T = params.temperature
    w1, w2 = math.exp(params.score[x[0], y[0]] / T), math.exp(params.score[x[1], y[0]] / T)
    assert abs(r["post_p"][0, 0] - w1 / (w1 + w2)) < 1e-14
    tau = 1 - 2 * sum(params.gap_open)
    assert abs(r["logz_h"] - math.log(tau * _g(1, params) * (e1 + e2))) < 1e-13


@pytest.mark.parametrize("xs,ys", [("AWK", "W"), ("DEF", "E"), ("GGG", "G")])
def test_3x1_two_gap_classes(params, xs, ys):
    # alignments: M X X (one run of 2, one M->M), X M X (two runs of 1, no
    # M->M), X X M (one run of 2, one M->M).  Exercises both gap classes.
    x, y = W.encode(xs), W.encode(ys)
    r = oracle.pair(x, y, params)
    e = _odds(params)
    tau = 1 - 2 * sum(params.gap_open)
    e1, e2, e3 = (e[x[k], y[0]] for k in range(3))
    a1, a2, a3 = tau * _g(2, params) * e1, _g(1, params) ** 2 * e2, tau * _g(2, params) * e3
    Z = a1 + a2 + a3
    for k, a in enumerate((a1, a2, a3)):
        assert abs(r["post_h"][k, 0] - a / Z) < 1e-14
    assert abs(r["logz_h"] - math.log(Z)) < 1e-13
    T, go, ge = params.temperature, params.pf_gap_open, params.pf_gap_extend
    w = [math.exp(params.score[x[k], y[0]] / T) for k in range(3)]
    b = [w[0] * math.exp((go + ge) / T), w[1] * math.exp(2 * go / T), w[2] * math.exp((go + ge) / T)]
    for k in range(3):
        assert abs(r["post_p"][k, 0] - b[k] / sum(b)) < 1e-14
    # and the transposed problem (1x3) gives the transposed answer
    rt = oracle.pair(y, x, params)
    np.testing.assert_allclose(rt["post"], r["post"].T, rtol=0, atol=1e-14)


def _gotoh(x, y, s, go, ge):
    """Textbook affine-gap global alignment (max-plus) restricted to no X-Y
    adjacency, begin/end as match; returns (best score, number of co-optimal
    alignments, match cells of one optimal alignment)."""
    m, n = len(x), len(y)
    NEG = -10 ** 9
    V = {k: [[NEG] * (n + 1) for _ in range(m + 1)] for k in "MXY"}
    C = {k: [[0] * (n + 1) for _ in range(m + 1)] for k in "MXY"}
    B = {k: [[None] * (n + 1) for _ in range(m + 1)] for k in "MXY"}
    V["M"][0][0], C["M"][0][0] = 0, 1

    def pick(cands):
        b = max(v for v, _, _ in cands)
        if b <= NEG // 2:
            return NEG, 0, None
        return b, sum(c for v, c, _ in cands if v == b), [k for v, _, k in cands if v == b][0]

    for i in range(m + 1):
        for j in range(n + 1):
            if i >= 1 and j >= 1:
                b, c, k = pick([(V[k][i - 1][j - 1], C[k][i - 1][j - 1], k) for k in "MXY"])
                if k is not None:
                    V["M"][i][j], C["M"][i][j], B["M"][i][j] = b + int(s[x[i - 1], y[j - 1]]), c, k
            if i >= 1:
                V["X"][i][j], C["X"][i][j], B["X"][i][j] = pick(
                    [(V["M"][i - 1][j] + go, C["M"][i - 1][j], "M"), (V["X"][i - 1][j] + ge, C["X"][i - 1][j], "X")])
            if j >= 1:
                V["Y"][i][j], C["Y"][i][j], B["Y"][i][j] = pick(
                    [(V["M"][i][j - 1] + go, C["M"][i][j - 1], "M"), (V["Y"][i][j - 1] + ge, C["Y"][i][j - 1], "Y")])
    bst, cnt, st = pick([(V[k][m][n], C[k][m][n], k) for k in "MXY"])
    cells = set()
    i, j = m, n
    while i > 0 or j > 0:
        prev = B[st][i][j]
        if st == "M":
            cells.add((i - 1, j - 1))
            i, j = i - 1, j - 1
        elif st == "X":
            i -= 1
        else:
            j -= 1
        st = prev
    return bst, cnt, cells


def test_zero_temperature_is_the_affine_gap_optimum(params):
    """T -> 0: the PF posterior becomes the indicator of the unique optimal
    (restricted Gotoh) alignment; integer scores give a gap of >= 1 score
    unit to the runner-up, i.e. a weight ratio <= exp(-1/T)."""
    fam = W.make_family(6, [14, 12, 15, 11, 13, 16], 123, r_sub=0.3, r_indel=0.1)
    T = 0.02
    p = params.copy(temperature=T)
    checked = 0
    for a in range(len(fam)):
        for b in range(a + 1, len(fam)):
            x, y = fam[a], fam[b]
            bst, cnt, cells = _gotoh(x, y, p.score, int(p.pf_gap_open), int(p.pf_gap_extend))
            if cnt != 1:
                continue
            r = oracle.pair(x, y, p)
            ind = np.zeros((len(x), len(y)))
            for (i, j) in cells:
                ind[i, j] = 1.0
            np.testing.assert_allclose(r["post_p"], ind, rtol=0, atol=1e-9)
            assert abs(r["logz_p"] - bst / T) < 1e-6
            checked += 1
    assert checked >= 5


@pytest.mark.parametrize("m,n", [(7, 9), (12, 15), (20, 11)])
def test_infinite_temperature_counts_alignments(params, m, n):
    """T -> infinity: every alignment weighs 1, so P(i,j) is the fraction of
    alignments through (i,j) = N(i-1,j-1) N(m-i,n-j) / N(m,n)."""
    p = params.copy(temperature=1e13)
    rng = np.random.default_rng(m * n)
    x = rng.integers(0, 20, m).astype(np.uint8)
    y = rng.integers(0, 20, n).astype(np.uint8)
    r = oracle.pair(x, y, p)
    N = bf.count_by_formula
    tot = N(m, n)
    exp = np.array([[N(i, j) * N(m - 1 - i, n - 1 - j) / tot for j in range(n)] for i in range(m)])
    np.testing.assert_allclose(r["post_p"], exp, rtol=0, atol=1e-10)
    assert abs(r["logz_p"] - math.log(tot)) < 1e-9


def test_equal_gap_classes_reduce_to_three_states(params):
    fam = W.c1_family()[:3]
    p5 = params.copy(gap_open=(0.02, 0.02), gap_extend=(0.5, 0.5))
    p3 = params.copy(gap_open=(0.04,), gap_extend=(0.5,))
    for a, b in [(0, 1), (1, 2)]:
        r5 = oracle.pair(fam[a][:40], fam[b][:50], p5)
        r3 = oracle.pair(fam[a][:40], fam[b][:50], p3)
        np.testing.assert_allclose(r5["post_h"], r3["post_h"], rtol=0, atol=1e-13)
        assert abs(r5["logz_h"] - r3["logz_h"]) < 1e-10


def test_one_class_hmm_equals_pf_under_mapping(params):
    """A one-class HMM equals a PF with w = e, o = delta (1-eps) tau^(-3/2),
    u = eps tau^(-1/2): W_H(A) / W_P(A) is the same constant for every
    alignment because #M = (m + n - sum of run lengths) / 2."""
    d, e = 0.03, 0.6
    tau = 1 - 2 * d
    T = 1.0
    p = params.copy(gap_open=(d,), gap_extend=(e,))
    sc = T * np.log(_odds(p))
    pf = params.copy(score=sc, pf_gap_open=T * math.log(d * (1 - e) * tau ** -1.5),
                     pf_gap_extend=T * math.log(e * tau ** -0.5), temperature=T)
    fam = W.c1_family()
    x, y = fam[0][:60], fam[3][:45]
    rh = oracle.pair(x, y, p)
    rp = oracle.pair(x, y, pf)
    np.testing.assert_allclose(rh["post_h"], rp["post_p"], rtol=0, atol=1e-12)
    m, n = len(x), len(y)
    const = (m + n) / 2 * math.log(tau) + math.log(tau)
    assert abs(rh["logz_h"] - (rp["logz_p"] + const)) < 1e-9
