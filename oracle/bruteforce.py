"""Posteriors by explicit enumeration of every alignment (tiny pairs only).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

This is the posterior written straight from its definition: the probability
that x_i is aligned with y_j is the total weight of the alignments that
contain the match column (i, j) divided by the total weight of all
alignments.  It enumerates alignments explicitly, so it shares no recurrence
with the dynamic programmes in ``qp_oracle.c`` and pins them.

Alignment space: monotone column sequences of M (match), X (x against a gap)
and Y (y against a gap) columns using every residue once, with no X column
adjacent to a Y column.  Begin and end count as match columns when counting
transitions.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import Callable, Iterator, List, Sequence, Tuple

import numpy as np

Column = Tuple[str, int, int]  # ('M', i, j) | ('X', i, -1) | ('Y', -1, j); 1-based


def alignments(m: int, n: int) -> Iterator[List[Column]]:
    """Every admissible alignment of lengths m and n."""
    out: List[Column] = []

    def rec(i: int, j: int, last: str):
        if i == m and j == n:
            yield list(out)
            return
        if i < m and j < n:
            out.append(("M", i + 1, j + 1))
            yield from rec(i + 1, j + 1, "M")
            out.pop()
        if i < m and last != "Y":
            out.append(("X", i + 1, -1))
            yield from rec(i + 1, j, "X")
            out.pop()
        if j < n and last != "X":
            out.append(("Y", -1, j + 1))
            yield from rec(i, j + 1, "Y")
            out.pop()

    yield from rec(0, 0, "M")


def count_by_formula(m: int, n: int) -> int:
    """Number of admissible alignments, counted combinatorially: choose k match
    columns (C(m,k) C(n,k) position choices); each of the k+1 segments between
    consecutive matches (and the two ends) holds unmatched residues of x or of
    y but not both, because an X run and a Y run would otherwise touch."""
    total = 0
    for k in range(0, min(m, n) + 1):
        total += _count_k(m, n, k)
    return total


def _count_k(m: int, n: int, k: int) -> int:
    # Distribute m-k unmatched x residues and n-k unmatched y residues over
    # k+1 segments such that no segment has both.  Count: choose which
    # segments carry x residues (a of them, each >= 1) and which carry y
    # residues (b of them, disjoint, each >= 1).
    ux, uy, s = m - k, n - k, k + 1
    tot = 0
    for a in range(0, s + 1):
        if (ux == 0) != (a == 0) or a > ux:
            continue
        wx = math.comb(ux - 1, a - 1) if a > 0 else 1
        for b in range(0, s - a + 1):
            if (uy == 0) != (b == 0) or b > uy:
                continue
            wy = math.comb(uy - 1, b - 1) if b > 0 else 1
            tot += math.comb(s, a) * math.comb(s - a, b) * wx * wy
    return tot


def _runs(cols: Sequence[Column]) -> List[Tuple[str, int]]:
    """Maximal gap runs as (kind, length)."""
    out: List[Tuple[str, int]] = []
    prev = "M"
    for c in cols:
        k = c[0]
        if k == "M":
            prev = "M"
            continue
        if prev == k:
            out[-1] = (k, out[-1][1] + 1)
        else:
            out.append((k, 1))
        prev = k
    return out


def hmm_weight(cols, x, y, e, tau, delta, eps):
    """Pair-HMM path weight (odds form), summed over the gap-class labels of
    each run: tau^(#M->M transitions) * prod e * prod_runs g(L),
    g(L) = sum_k delta_k eps_k^(L-1) (1 - eps_k).  Works with floats or
    Fractions."""
    n_m = sum(1 for c in cols if c[0] == "M")
    rs = _runs(cols)
    w = tau ** (n_m + 1 - len(rs))
    for c in cols:
        if c[0] == "M":
            w = w * e[x[c[1] - 1]][y[c[2] - 1]]
    for (_, L) in rs:
        g = 0
        for d, ep in zip(delta, eps):
            g = g + d * ep ** (L - 1) * (1 - ep)
        w = w * g
    return w


def pf_log_weight(cols, x, y, score, g_open, g_ext, T):
    """log of the partition-function weight exp(score(A)/T)."""
    s = 0.0
    for c in cols:
        if c[0] == "M":
            s += score[x[c[1] - 1]][y[c[2] - 1]]
    for (_, L) in _runs(cols):
        s += g_open + (L - 1) * g_ext
    return s / T


def posterior_from_weights(m: int, n: int, weighted: List[Tuple[List[Column], object]]):
    """P(i,j) = sum of weights of alignments containing M(i,j) / total."""
    Z = sum(w for _, w in weighted)
    P = [[0 for _ in range(n)] for _ in range(m)]
    for cols, w in weighted:
        for c in cols:
            if c[0] == "M":
                P[c[1] - 1][c[2] - 1] = P[c[1] - 1][c[2] - 1] + w
    return [[v / Z for v in row] for row in P], Z


def hmm_posterior(x, y, joint, delta, eps, exact: bool = False):
    """Brute-force pair-HMM posterior.  With ``exact`` the joint and gap
    parameters must be Fractions (or ints) and the result is exact."""
    m, n = len(x), len(y)
    A = 20
    if exact:
        J = [[Fraction(joint[a][b]) for b in range(A)] for a in range(A)]
        qx = [sum(J[a]) for a in range(A)]
        qy = [sum(J[a][b] for a in range(A)) for b in range(A)]
        e = [[J[a][b] / (qx[a] * qy[b]) if qx[a] and qy[b] else Fraction(0) for b in range(A)] for a in range(A)]
        d = [Fraction(v) for v in delta]
        ep = [Fraction(v) for v in eps]
        tau = 1 - 2 * sum(d)
    else:
        J = np.asarray(joint, dtype=np.float64)
        qx, qy = J.sum(1), J.sum(0)
        e = (J / np.outer(qx, qy)).tolist()
        d, ep = list(map(float, delta)), list(map(float, eps))
        tau = 1.0 - 2.0 * sum(d)
    weighted = [(cols, hmm_weight(cols, x, y, e, tau, d, ep)) for cols in alignments(m, n)]
    return posterior_from_weights(m, n, weighted)


def pf_posterior(x, y, score, g_open, g_ext, T):
    """Brute-force partition-function posterior (floats, max-shifted)."""
    m, n = len(x), len(y)
    al = list(alignments(m, n))
    lw = [pf_log_weight(c, x, y, score, g_open, g_ext, T) for c in al]
    mx = max(lw)
    weighted = [(c, math.exp(v - mx)) for c, v in zip(al, lw)]
    P, Z = posterior_from_weights(m, n, weighted)
    return P, mx + math.log(Z)


def mea_brute(P) -> float:
    """Maximum over monotone matchings (strictly increasing in i and j) of the
    summed entries, by recursion over cells."""
    P = np.asarray(P, dtype=np.float64)
    m, n = P.shape
    best = 0.0

    def rec(i0: int, j0: int, acc: float):
        nonlocal best
        if acc > best:
            best = acc
        for i in range(i0, m):
            for j in range(j0, n):
                rec(i + 1, j + 1, acc + P[i, j])

    rec(0, 0, 0.0)
    return best
