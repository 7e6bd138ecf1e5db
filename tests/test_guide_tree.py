"""Guide tree (weighted UPGMA) and tree-guided distance: the oracle against
what the definitions fix, then the library (host code, no device) against
the oracle, exactly."""
import numpy as np
import pytest

from oracle import tree as T


@pytest.fixture(scope="module")
def B():
    from paper_1512_07437_amd import binding
    return binding


def _condensed(M):
    n = len(M)
    return np.array([M[i][j] for i in range(n) for j in range(i + 1, n)], dtype=np.float64)


def _clusters(joins, n):
    """Every join as the set of sequences under it."""
    members = {i: frozenset([i]) for i in range(n)}
    out = []
    for k, (a, b) in enumerate(joins):
        members[n + k] = members[a] | members[b]
        out.append(members[n + k])
    return out


def _random_ultrametric(rng, n):
    """Random binary tree with strictly increasing join heights; distances are
    twice the height of the lowest common join."""
    members = {i: [i] for i in range(n)}
    live = list(range(n))
    M = np.zeros((n, n))
    h = 0.0
    clusters = []
    for k in range(n - 1):
        a, b = rng.choice(live, 2, replace=False)
        h += float(rng.integers(1, 9))  # exact in binary
        for x in members[a]:
            for y in members[b]:
                M[x, y] = M[y, x] = 2.0 * h
        members[n + k] = members[a] + members[b]
        live.remove(a)
        live.remove(b)
        live.append(n + k)
        clusters.append((frozenset(members[n + k]), h))
    return M, clusters


# ---------------------------------------------------------------- oracle pins
@pytest.mark.parametrize("seed", range(5))
def test_oracle_recovers_ultrametric_tree(seed):
    """On ultrametric distances every join is exact: the oracle returns the
    generating tree (same clusters, same heights)."""
    rng = np.random.default_rng(seed)
    n = 12
    M, truth = _random_ultrametric(rng, n)
    joins, heights = T.wpgma(_condensed(M), n)
    got = sorted(zip(_clusters(joins, n), heights), key=lambda c: (c[1], sorted(c[0])))
    want = sorted(truth, key=lambda c: (c[1], sorted(c[0])))
    assert got == want


def test_oracle_hand_example_weighted_not_size_weighted():
    """Four sequences, worked by hand: join (0,1) at 2, then (2, {0,1}) at 4;
    the last distance is the plain mean (10 + 6)/2 = 8 (height 4), where the
    size-weighted mean would give (2*10 + 6)/3."""
    M = [[0, 2, 4, 10],
         [2, 0, 4, 10],
         [4, 4, 0, 6],
         [10, 10, 6, 0]]
    joins, heights = T.wpgma(_condensed(M), 4)
    assert joins == [(0, 1), (2, 4), (3, 5)]
    assert heights == [1.0, 2.0, 4.0]
    # subtree under the first common join: {0,1} has 3 nodes, {0,1,2} 5, all 7
    assert T.tree_distance(joins, 4) == [3, 5, 7, 5, 7, 7]


def test_oracle_heights_never_decrease():
    """Joining the two closest clusters by the plain mean never creates a
    closer pair, so join heights are non-decreasing."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        n = int(rng.integers(2, 15))
        pts = rng.normal(size=(n, 3))
        M = np.sqrt(((pts[:, None] - pts[None]) ** 2).sum(-1))
        _, heights = T.wpgma(_condensed(M), n)
        assert all(b >= a for a, b in zip(heights, heights[1:]))


def test_oracle_tree_distance_caterpillar():
    """A chain (0,1), then 2, then 3 ...: sequences 0 and 1 share a cherry (3
    nodes); 0 and k (k >= 2) first meet in the join holding k+1 sequences."""
    n = 7
    joins = [(0, 1)] + [(k, n + k - 2) for k in range(2, n)]
    td = T.tree_distance(joins, n)
    for j in range(1, n):
        want = 3 if j == 1 else 2 * (j + 1) - 1
        assert td[T.pair_index(0, j, n)] == want


# ---------------------------------------------------- library vs the oracle
@pytest.mark.parametrize("seed", range(12))
def test_library_equals_oracle(B, seed):
    """Same joins, bit-identical heights and the same tree distances; half the
    cases draw distances from a few values, so ties are frequent."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 40))
    P = n * (n - 1) // 2
    dist = (rng.integers(0, 4, size=P).astype(np.float64) if seed % 2 else rng.uniform(0, 1, size=P))
    joins_o, heights_o = T.wpgma(dist, n)
    joins, heights = B.guide_tree(dist, n)
    assert [tuple(map(int, j)) for j in joins] == joins_o
    assert heights.tolist() == heights_o
    assert B.tree_distance(joins, n).tolist() == T.tree_distance(joins_o, n)


def test_library_on_a_family(B):
    """The distances of a synthetic family (EA distances are in [0, 1]): the
    library's tree is the oracle's."""
    rng = np.random.default_rng(3)
    n = 30
    dist = np.round(rng.uniform(0.2, 0.9, size=n * (n - 1) // 2), 3)
    joins, heights = B.guide_tree(dist, n)
    jo, ho = T.wpgma(dist, n)
    assert [tuple(map(int, j)) for j in joins] == jo and heights.tolist() == ho


def test_library_edge_cases_and_errors(B):
    j, h = B.guide_tree(np.zeros(0), 1)
    assert j.shape == (0, 2) and h.shape == (0,)
    assert B.tree_distance(j, 1).shape == (0,)
    j, h = B.guide_tree(np.array([0.5]), 2)
    assert j.tolist() == [[0, 1]] and h.tolist() == [0.25]
    assert B.tree_distance(j, 2).tolist() == [3]
    with pytest.raises(B.QpError) as e:
        B.guide_tree(np.array([0.1, np.nan, 0.3]), 3)
    assert e.value.status == B.QP_EINVAL
    with pytest.raises(B.QpError) as e:
        B.tree_distance(np.array([[0, 1], [0, 3]]), 3)  # 0 joined twice
    assert e.value.status == B.QP_EINVAL
    with pytest.raises(B.QpError) as e:
        B.tree_distance(np.array([[0, 1], [2, 5]]), 3)  # 5 does not exist yet
    assert e.value.status == B.QP_EINVAL
    assert B.lib.qp_guide_tree(None, 0, None, None) == B.QP_EINVAL


# --------------------------------------------- planted mistakes in the oracle
def _linkage(dist, n, rule):
    """The oracle's join loop with another merge rule (a planted mistake)."""
    D = {}
    for i in range(n):
        for j in range(i + 1, n):
            D[(i, j)] = float(dist[T.pair_index(i, j, n)])
    size = {i: 1 for i in range(n)}

    def get(a, b):
        return D[(a, b)] if a < b else D[(b, a)]

    active = list(range(n))
    joins, heights = [], []
    for step in range(n - 1):
        d, a, b = min((get(a, b), a, b) for a in active for b in active if a < b)
        made = n + step
        for x in active:
            if x != a and x != b:
                D[(x, made)] = rule(get(a, x), get(b, x), size[a], size[b])
        size[made] = size[a] + size[b]
        active.remove(a)
        active.remove(b)
        active.append(made)
        joins.append((a, b))
        heights.append(d / 2.0)
    return joins, heights


@pytest.mark.parametrize("name,rule", [
    ("size-weighted mean (UPGMA)", lambda da, db, na, nb: (na * da + nb * db) / (na + nb)),
    ("single linkage", lambda da, db, na, nb: min(da, db)),
    ("complete linkage", lambda da, db, na, nb: max(da, db)),
    ("mean without halving", lambda da, db, na, nb: da + db),
])
def test_hand_example_catches_other_merge_rules(name, rule):
    """Each plausible wrong merge rule changes the hand-worked heights."""
    M = [[0, 2, 4, 10], [2, 0, 4, 10], [4, 4, 0, 6], [10, 10, 6, 0]]
    _, heights = _linkage(_condensed(M), 4, rule)
    assert heights != [1.0, 2.0, 4.0], name
    _, ok = _linkage(_condensed(M), 4, lambda da, db, na, nb: (da + db) / 2.0)
    assert ok == [1.0, 2.0, 4.0]


def test_caterpillar_catches_counting_only_sequences():
    """Counting the sequences under the common join instead of all its nodes
    (or the path between the two) gives other numbers on the chain."""
    n = 7
    joins = [(0, 1)] + [(k, n + k - 2) for k in range(2, n)]
    td = T.tree_distance(joins, n)
    leaves_only = [2 if j == 1 else j + 1 for j in range(1, n)]
    path_nodes = [3] + [j + 2 for j in range(2, n)]  # 0 .. up to the join .. down to j
    got = [td[T.pair_index(0, j, n)] for j in range(1, n)]
    assert got != leaves_only and got != path_nodes
