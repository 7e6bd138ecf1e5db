"""Pins of the selective-consistency oracle (``oracle/consistency.py``).

- Full consistency as one block-matrix product: with h = 1 and every third
  sequence selected, the relaxation must equal (1/k) (M M)_xy where M is the
  block matrix of all posterior matrices with identity blocks on the
  diagonal -- an independent statement of "average over z of S_xz S_zy".
- A hand-worked three-sequence family (every number below is written out).
- The amplification coefficient and the tree-guided selection on a
  four-sequence tree worked by hand.
- Invariants on real oracle posteriors: row and column sums <= 1, entries
  at or above the threshold, the transpose relation S'_yx = S'_xy^T.
- Planted mistakes in the oracle's source fail these pins.
"""
import os
import types

import numpy as np
import pytest

import oracle
from oracle import consistency as C
from oracle import tree as OT
from paper_1512_07437_amd import workload as W

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "consistency.py")


def _random_family(rng, k, lo=2, hi=5, density=0.5):
    """Random nonnegative matrices with row and column sums <= 1 (any
    matrices serve the algebraic pins)."""
    lens = rng.integers(lo, hi + 1, size=k)
    S = {}
    for x in range(k):
        for y in range(x + 1, k):
            a = rng.random((lens[x], lens[y])) * (rng.random((lens[x], lens[y])) < density)
            a /= max(1.0, a.sum(axis=1).max(), a.sum(axis=0).max())
            S[(x, y)] = a
    return lens, S


def _block(S, lens, k):
    off = np.concatenate([[0], np.cumsum(lens)])
    M = np.zeros((off[-1], off[-1]))
    for x in range(k):
        M[off[x]:off[x + 1], off[x]:off[x + 1]] = np.eye(lens[x])
        for y in range(k):
            if x != y:
                M[off[x]:off[x + 1], off[y]:off[y + 1]] = C.get(S, x, y)
    return M, off


def _check_full_consistency(mod, seed):
    rng = np.random.default_rng(seed)
    k = 5
    lens, S = _random_family(rng, k)
    tdist = [1] * (k * (k - 1) // 2)
    out = mod.relax_pass(S, k, tdist, T=1e9, h=1.0, thresh=0.0)
    M, off = _block(S, lens, k)
    MM = M @ M / k
    for (x, y), v in out.items():
        np.testing.assert_allclose(v, MM[off[x]:off[x + 1], off[y]:off[y + 1]], rtol=0, atol=1e-14)


def test_full_consistency_is_block_product():
    for seed in range(4):
        _check_full_consistency(C, seed)


def _three_sequence_family():
    S = {(0, 1): np.array([[0.5, 0.1], [0.2, 0.6]]),
         (0, 2): np.array([[0.7], [0.2]]),
         (1, 2): np.array([[0.4], [0.3]])}
    return S


def _check_three_sequences(mod):
    # k = 3, every z selected: h_xy = 1 + (3 - 1) * 1/1 = 3, so
    # S'_xy = (6 S_xy + S_xz S_zy) / 7, entries below 0.15 dropped.
    S = _three_sequence_family()
    out = mod.relax_pass(S, 3, [1, 1, 1], T=10, h=3.0, thresh=0.15)
    # S_02 S_21 = [[.7*.4, .7*.3], [.2*.4, .2*.3]] = [[.28, .21], [.08, .06]]
    # 6 S_01 + that = [[3.28, 0.81], [1.28, 3.66]]; / 7; 0.81/7 < 0.15 dropped
    np.testing.assert_allclose(out[(0, 1)], [[3.28 / 7, 0.0], [1.28 / 7, 3.66 / 7]], rtol=0, atol=1e-15)
    # S_01 S_12 = [[.5*.4 + .1*.3], [.2*.4 + .6*.3]] = [[.23], [.26]]
    np.testing.assert_allclose(out[(0, 2)], [[(4.2 + 0.23) / 7], [(1.2 + 0.26) / 7]], rtol=0, atol=1e-15)
    # S_10 S_02 = S_01^T S_02 = [[.5*.7 + .2*.2], [.1*.7 + .6*.2]] = [[.39], [.19]]
    np.testing.assert_allclose(out[(1, 2)], [[(2.4 + 0.39) / 7], [(1.8 + 0.19) / 7]], rtol=0, atol=1e-15)


def test_three_sequences_by_hand():
    _check_three_sequences(C)


def _four_tree():
    # (((0, 1), 2), 3): joins 0+1 -> 4, 4+2 -> 5, 5+3 -> 6
    joins = [(0, 1), (2, 4), (3, 5)]
    return OT.tree_distance(joins, 4)


def _check_four_tree(mod):
    tdist = _four_tree()
    # subtree node counts by hand: {0,1}: 3 nodes; {0,1,2}: 5; whole tree: 7
    assert [tdist[OT.pair_index(i, j, 4)] for (i, j) in ((0, 1), (0, 2), (1, 2), (0, 3), (2, 3))] == [3, 5, 5, 7, 7]
    assert mod.selected(tdist, 4, 0, 1, 5) == [2]
    assert mod.selected(tdist, 4, 2, 3, 5) == []
    assert mod.selected(tdist, 4, 0, 1, 7) == [2, 3]
    # one of the two other sequences selected: h_01 = 1 + (3 - 1) * 1/2 = 2
    assert mod.amplification(1, 4, 3.0) == 2.0
    S = {(a, b): np.array([[v]]) for (a, b), v in {(0, 1): 0.6, (0, 2): 0.5, (1, 2): 0.4, (0, 3): 0.3,
                                                   (1, 3): 0.2, (2, 3): 0.9}.items()}
    out = mod.relax_pass(S, 4, tdist, T=5, h=3.0, thresh=0.01)
    # (4 * 0.6 + 0.5 * 0.4) / (4 + 1)
    assert abs(out[(0, 1)][0, 0] - 0.52) < 1e-15
    # nothing selected for (2, 3): h_23 = 1 and S' = (2 S) / 2 = S
    assert abs(out[(2, 3)][0, 0] - 0.9) < 1e-15
    # (0, 2): z = 1 has max(d01, d12) = 5 -> selected; z = 3 has 7 -> not
    assert abs(out[(0, 2)][0, 0] - (4 * 0.5 + 0.6 * 0.4) / 5) < 1e-15


def test_selection_and_amplification_by_hand():
    _check_four_tree(C)


def test_passes_per_family_size():
    assert C.passes_for(10) == 2 and C.passes_for(49) == 2 and C.passes_for(50) == 1 and C.passes_for(500) == 1


def test_invariants_on_oracle_posteriors(params):
    fam = W.c1_family()[:5]
    k = len(fam)
    thresh = 0.01
    S0 = {}
    dist = []
    for x in range(k):
        for y in range(x + 1, k):
            r = oracle.pair(fam[x], fam[y], params, per_model=False)
            p = r["post"].copy()
            p[p < thresh] = 0.0
            S0[(x, y)] = p
            dist.append(1.0 - r["ea"])
    joins, _ = OT.wpgma(dist, k)
    tdist = OT.tree_distance(joins, k)
    out = C.consistency(S0, k, tdist, T=7, h=3.0, passes=2, thresh=thresh)
    for (x, y), v in out.items():
        assert v.shape == S0[(x, y)].shape
        assert v.sum(axis=1).max() <= 1 + 1e-12 and v.sum(axis=0).max() <= 1 + 1e-12
        assert np.all((v == 0) | (v >= thresh))
    # the relaxation of (y, x) is the transpose of that of (x, y)
    S1 = C.relax_pass(S0, k, tdist, T=7, h=3.0, thresh=0.0)
    for (x, y) in S1:
        Z = C.selected(tdist, k, y, x, 7)
        hyx = C.amplification(len(Z), k, 3.0)
        acc = 2 * hyx * C.get(S0, y, x)
        for z in Z:
            acc = acc + C.get(S0, y, z) @ C.get(S0, z, x)
        np.testing.assert_allclose(acc / (2 * hyx + len(Z)), S1[(x, y)].T, rtol=0, atol=1e-14)


MUTANTS = {
    "own_term_once": ("acc = 2.0 * hxy * S[(x, y)]", "acc = hxy * S[(x, y)]"),
    "norm_without_own": ("acc = acc / (2.0 * hxy + len(Z))", "acc = acc / (len(Z) + 1)"),
    "no_transpose": ("return S[(a, b)] if a < b else S[(b, a)].T", "return S[(a, b)] if a < b else S[(b, a)]"),
    "selection_sum": ("if max(dxz, dyz) <= T:", "if dxz + dyz <= T:"),
    "amplification_flat": ("return 1.0 if k <= 2 else 1.0 + (h - 1.0) * n_sel / (k - 2)", "return h"),
    "product_order": ("acc = acc + get(S, x, z) @ get(S, z, y)", "acc = acc + (get(S, z, y).T @ get(S, x, z).T).T * 0.5"),
}


def _mutant(name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert old in src, "mutation anchor not found: " + name
    mod = types.ModuleType("consistency_" + name)
    mod.__dict__["__package__"] = "oracle"
    exec(compile(src.replace(old, new, 1), SRC, "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistakes(name):
    mod = _mutant(name)
    failures = 0
    for check in (lambda: _check_full_consistency(mod, 0), lambda: _check_three_sequences(mod),
                  lambda: _check_four_tree(mod)):
        try:
            check()
        except (AssertionError, ValueError):  # a wrong value, or operands that no longer fit
            failures += 1
    assert failures > 0, "mutant %s passed every pin" % name
