"""Guaranteed output size and the threshold for a memory budget (host logic,
no device): the bound is the row count times the per-row cap, and the
threshold returned is the smallest one whose bound fits."""
import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def B():
    from paper_1512_07437_amd import binding
    return binding


def _bound(lens, thresh, pairs=None):
    t = float(np.float32(thresh))
    cap = math.floor(1.0 / t) + 1
    if pairs is None:
        pairs = [(i, j) for i in range(len(lens)) for j in range(i + 1, len(lens))]
    return sum(int(lens[i]) * min(int(lens[j]), cap) for i, j in pairs)


@pytest.mark.parametrize("thresh", [1.0, 0.5, 0.2, 0.01, 0.003, 1e-4])
def test_bound_formula(B, thresh):
    rng = np.random.default_rng(1)
    lens = rng.integers(1, 400, size=23).astype(np.int32)
    assert B.output_bound(lens, thresh) == _bound(lens, thresh)
    pi = np.array([0, 5, 7, 22], dtype=np.int32)
    pj = np.array([1, 3, 20, 2], dtype=np.int32)
    assert B.output_bound(lens, thresh, pi, pj) == _bound(lens, thresh, list(zip(pi, pj)))


def test_bound_holds_for_every_row():
    """The per-row cap is what any row can hold: posteriors of a row sum to at
    most one (checked on oracle rows at several thresholds)."""
    import oracle
    from paper_1512_07437_amd import workload as W
    fam = W.c1_family()[:3]
    mp = W.make_params(0)
    for i, j in ((0, 1), (0, 2), (1, 2)):
        post = oracle.pair(fam[i], fam[j], mp, per_model=False)["post"]
        for t in (0.5, 0.1, 0.01, 0.001):
            cap = math.floor(1.0 / t) + 1
            assert int((post >= t).sum(axis=1).max()) <= min(post.shape[1], cap)


@pytest.mark.parametrize("seed", range(6))
def test_threshold_for_budget_is_smallest(B, seed):
    rng = np.random.default_rng(seed)
    lens = rng.integers(5, 300, size=int(rng.integers(3, 30))).astype(np.int32)
    dense = _bound(lens, 1e-30)
    floor2 = _bound(lens, 1.0)
    budget = int(rng.integers(floor2, dense + 1))
    t = B.threshold_for_budget(lens, budget)
    assert 0.0 < t <= 1.0
    assert B.output_bound(lens, t) <= budget
    lower = float(np.nextafter(np.float32(t), np.float32(0)))
    if B.output_bound(lens, t) < dense:  # not saturated: one float lower no longer fits
        assert B.output_bound(lens, lower) > budget


def test_threshold_for_budget_limits(B):
    lens = np.array([100, 120, 90], dtype=np.int32)
    with pytest.raises(B.QpError) as e:
        B.threshold_for_budget(lens, _bound(lens, 1.0) - 1)
    assert e.value.status == B.QP_ENOSPC
    t = B.threshold_for_budget(lens, 10 ** 12)  # everything fits: rows first keep every column
    assert B.output_bound(lens, t) == _bound(lens, 1e-30)
    with pytest.raises(B.QpError):
        B.output_bound(lens, 0.0)
    with pytest.raises(B.QpError):
        B.output_bound(np.array([100, 0], dtype=np.int32), 0.01)
    with pytest.raises(B.QpError):
        B.output_bound(lens, 0.01, [0], [0])
