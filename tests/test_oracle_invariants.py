"""Invariants of the posterior that hold at any size (FP64 oracle).

- every posterior is in [0, 1]; row and column sums are <= 1 (each residue is
  matched at most once in any alignment);
- forward and backward totals agree;
- the model is symmetric in x and y: P(y, x) = P(x, y)^T;
- the model is symmetric under reversing both sequences (begin and end are
  both match states): P(rev x, rev y)(i, j) = P(x, y)(m-1-i, n-1-j);
- the thresholded CSR keeps at most floor(1/thresh) entries per row;
- 0 <= EA <= 1 and EA >= max P / min(m, n).
"""
import numpy as np
import pytest

import oracle
from paper_1512_07437_amd import workload as W


@pytest.fixture(scope="module")
def fam():
    return W.c1_family()


@pytest.mark.parametrize("a,b", [(0, 1), (2, 5), (3, 7)])
def test_bounds_and_totals(fam, params, a, b):
    r = oracle.pair(fam[a], fam[b], params)
    for key in ("post", "post_h", "post_p"):
        P = r[key]
        assert P.min() >= 0.0 and P.max() <= 1.0 + 1e-12
        assert P.sum(axis=1).max() <= 1.0 + 1e-12
        assert P.sum(axis=0).max() <= 1.0 + 1e-12
    assert abs(r["logz_h"] - r["logz_h_bwd"]) <= 1e-12 * abs(r["logz_h"])
    assert abs(r["logz_p"] - r["logz_p_bwd"]) <= 1e-12 * abs(r["logz_p"])
    assert 0.0 <= r["ea"] <= 1.0
    assert r["ea"] >= r["post"].max() / min(len(fam[a]), len(fam[b])) - 1e-15


def test_symmetry(fam, params):
    r = oracle.pair(fam[1], fam[4], params)
    rt = oracle.pair(fam[4], fam[1], params)
    np.testing.assert_allclose(rt["post"], r["post"].T, rtol=0, atol=1e-13)
    assert abs(r["logz_h"] - rt["logz_h"]) < 1e-10
    assert abs(r["ea"] - rt["ea"]) < 1e-13


def test_reversal(fam, params):
    x, y = fam[2][:70], fam[6][:55]
    r = oracle.pair(x, y, params)
    rr = oracle.pair(x[::-1].copy(), y[::-1].copy(), params)
    np.testing.assert_allclose(rr["post"], r["post"][::-1, ::-1], rtol=0, atol=1e-13)
    assert abs(r["logz_h"] - rr["logz_h"]) < 1e-10
    assert abs(r["logz_p"] - rr["logz_p"]) < 1e-10


@pytest.mark.parametrize("thresh", [0.01, 0.05, 0.3])
def test_csr_shape(fam, params, thresh):
    r = oracle.pair(fam[0], fam[3], params)
    rp, col, val = oracle.to_csr(r["post"], thresh)
    assert rp[0] == 0 and rp[-1] == len(col) == len(val)
    assert np.all(np.diff(rp) <= int(1.0 / thresh))
    assert np.all(val >= thresh)
    for i in range(len(rp) - 1):
        c = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0)
    # nothing above the threshold is dropped
    assert int((r["post"] >= thresh).sum()) == len(col)


def test_identical_sequences_concentrate_on_the_diagonal(params):
    x = W.c1_family()[0]
    r = oracle.pair(x, x, params)
    d = np.diag(r["post"])
    assert d.mean() > 0.9
    assert r["ea"] > 0.9


def test_unrelated_sequences_are_diffuse(params):
    rng = np.random.default_rng(4)
    x, y = (rng.integers(0, 20, 90).astype(np.uint8) for _ in range(2))
    r = oracle.pair(x, y, params)
    rel = oracle.pair(W.c1_family()[0], W.c1_family()[1], params)
    assert r["ea"] < rel["ea"]
