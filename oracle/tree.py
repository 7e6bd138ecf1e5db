"""Guide-tree oracle: weighted UPGMA and the tree-guided distance.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``); shares no code with
the library.

What is computed (paper: Methods, opening paragraph -- the distances of the
posterior stage go into weighted UPGMA to build the guide tree; "Selective
consistency" -- the tree-guided distance of two sequences is the number of
nodes of the smallest subtree that holds both).

Weighted UPGMA (WPGMA, Sneath and Sokal): repeatedly join the two closest
clusters; the distance from the joined cluster to any other cluster is the
plain mean of the two joined clusters' distances to it, whatever their sizes
(the size-weighted mean would be UPGMA).  Ties between equal distances go to
the pair with the smaller smaller id, then the smaller larger id; sequence i
has id i, the cluster made at step k has id n + k.

The smallest subtree holding x and y is the subtree under their lowest common
ancestor; its nodes are counted by walking it.

Pins (tests): exact recovery of an ultrametric tree, a hand-worked example
on which weighted and size-weighted UPGMA differ, non-decreasing join
heights, and hand-counted subtree sizes on small trees.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple


def pair_index(i: int, j: int, n: int) -> int:
    return i * n - i * (i + 1) // 2 + (j - i - 1)


def wpgma(dist: Sequence[float], n: int) -> Tuple[List[Tuple[int, int]], List[float]]:
    """Joins (smaller id, larger id) and join heights (half the distance)."""
    D: Dict[Tuple[int, int], float] = {}
    for i in range(n):
        for j in range(i + 1, n):
            D[(i, j)] = float(dist[pair_index(i, j, n)])

    def get(a: int, b: int) -> float:
        return D[(a, b)] if a < b else D[(b, a)]

    active = list(range(n))
    joins: List[Tuple[int, int]] = []
    heights: List[float] = []
    for step in range(n - 1):
        d, a, b = min((get(a, b), a, b) for a in active for b in active if a < b)
        made = n + step
        for x in active:
            if x != a and x != b:
                D[(x, made)] = (get(a, x) + get(b, x)) / 2.0
        active.remove(a)
        active.remove(b)
        active.append(made)
        joins.append((a, b))
        heights.append(d / 2.0)
    return joins, heights


def tree_distance(joins: Sequence[Tuple[int, int]], n: int) -> List[int]:
    """For every pair i < j in pair order: nodes of the subtree under the
    lowest common ancestor of i and j."""
    parent: Dict[int, int] = {}
    children: Dict[int, Tuple[int, int]] = {}
    for step, (a, b) in enumerate(joins):
        parent[a] = parent[b] = n + step
        children[n + step] = (a, b)

    def ancestors(x: int) -> List[int]:
        out = [x]
        while out[-1] in parent:
            out.append(parent[out[-1]])
        return out

    def count(node: int) -> int:
        if node not in children:
            return 1
        a, b = children[node]
        return 1 + count(a) + count(b)

    out = [0] * (n * (n - 1) // 2)
    for i in range(n):
        up_i = ancestors(i)
        for j in range(i + 1, n):
            on_path = set(ancestors(j))
            lca = next(v for v in up_i if v in on_path)
            out[pair_index(i, j, n)] = count(lca)
    return out
