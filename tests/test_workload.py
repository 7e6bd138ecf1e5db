"""The seeded input generator: determinism, shapes, and the evolution rates."""
import numpy as np

from paper_1512_07437_amd import workload as W


def test_params_are_valid():
    p = W.make_params(0)
    assert abs(p.joint.sum() - 1.0) < 1e-12
    assert np.allclose(p.joint, p.joint.T)
    assert np.allclose(p.score, p.score.T)
    assert np.all(p.score == np.round(p.score))
    assert 1 - 2 * sum(p.gap_open) > 0


def test_determinism():
    a, b = W.c1_family(), W.c1_family()
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert W.make_params(0).joint.tobytes() == W.make_params(0).joint.tobytes()


def test_c1_shape():
    f = W.c1_family()
    assert len(f) == 8
    assert all(80 <= len(s) <= 120 for s in f)
    assert all(s.dtype == np.uint8 and s.max() < 20 for s in f)


def test_c2_shape_and_sample():
    f = W.c2_family()
    assert len(f) == 200 and all(250 <= len(s) <= 350 for s in f)
    s = W.c2_sample()
    assert len(s) == 200 and len(np.unique(s)) == 200 and s.max() < 19900


def test_substitution_rate_matches():
    p = W.make_params(0)
    q = W.background(p)
    rng = np.random.default_rng(0)
    root = rng.choice(20, size=20000, p=q).astype(np.uint8)
    leaf = W.evolve(root, rng, q, W.substitution_matrix(0), 0.3, 0.0)
    assert len(leaf) == len(root)
    frac = float(np.mean(leaf != root))
    assert abs(frac - 0.3) < 0.02  # substituted residues always change (zero diagonal)


def test_pair_index_roundtrip():
    n = 9
    k = 0
    for i in range(n):
        for j in range(i + 1, n):
            assert W.pair_index(i, j, n) == k
            assert W.pair_of_index(k, n) == (i, j)
            k += 1
