"""Selective-consistency oracle: relaxation of the sparse posterior matrices
through third sequences chosen by the guide tree.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``); shares no code with
the library.

What is computed (paper: Methods, "Selective consistency" -- a posterior
matrix S_xy is relaxed through a third sequence z when a function of the
tree-guided distances d_xz, d_yz meets a condition, the variant kept being
max(d_xz, d_yz) <= T with T about 200; the original S_xy is amplified by a
coefficient h_xy in [1, h], h = 3, set per matrix from the number of
relaxations it receives; "Other algorithmic improvements" -- two passes for
families under 50 sequences, one otherwise).  The relaxation itself is the
one the method inherits (consistency transformation of the probabilistic
aligners it descends from): S'_xy averages, over sequences z, the products
S_xz S_zy, where z = x and z = y contribute S_xy itself (S_xx is the
identity).  Readings fixed here, where the paper gives no formula:

  Z_xy  = { z not in {x, y} : max(d_xz, d_yz) <= T }
  h_xy  = 1 + (h - 1) |Z_xy| / (k - 2)   (k sequences; 1 when k = 2)
  S'_xy = (2 h_xy S_xy + sum_{z in Z_xy} S_xz S_zy) / (2 h_xy + |Z_xy|)

then entries below the sparsity threshold are dropped.  With h = 1 and every
z selected this is the full consistency transformation
S'_xy = (1/k) sum_{z=1..k} S_xz S_zy.  S_ab for a > b is S_ba transposed.
Each pass relaxes every pair from the previous pass's matrices.

Plain dense numpy: every matrix is a dense m x n array with the dropped
entries at zero.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np

from .tree import pair_index


def get(S: Dict[Tuple[int, int], np.ndarray], a: int, b: int) -> np.ndarray:
    """S_ab for a != b from the i < j store (transposed when a > b)."""
    return S[(a, b)] if a < b else S[(b, a)].T


def selected(tdist: Sequence[int], k: int, x: int, y: int, T: float) -> List[int]:
    """Z_xy: the third sequences whose tree-guided distances to x and to y are
    both at most T (tdist in pair order)."""
    out = []
    for z in range(k):
        if z == x or z == y:
            continue
        dxz = tdist[pair_index(min(x, z), max(x, z), k)]
        dyz = tdist[pair_index(min(y, z), max(y, z), k)]
        if max(dxz, dyz) <= T:
            out.append(z)
    return out


def amplification(n_sel: int, k: int, h: float) -> float:
    """h_xy: 1 with no relaxation, h when every other sequence relaxes S_xy."""
    return 1.0 if k <= 2 else 1.0 + (h - 1.0) * n_sel / (k - 2)


def relax_pass(S: Dict[Tuple[int, int], np.ndarray], k: int, tdist: Sequence[int], T: float, h: float,
               thresh: float) -> Dict[Tuple[int, int], np.ndarray]:
    """One pass over every pair x < y."""
    out = {}
    for x in range(k):
        for y in range(x + 1, k):
            Z = selected(tdist, k, x, y, T)
            hxy = amplification(len(Z), k, h)
            acc = 2.0 * hxy * S[(x, y)]
            for z in Z:
                acc = acc + get(S, x, z) @ get(S, z, y)
            acc = acc / (2.0 * hxy + len(Z))
            acc[acc < thresh] = 0.0
            out[(x, y)] = acc
    return out


def consistency(S0: Dict[Tuple[int, int], np.ndarray], k: int, tdist: Sequence[int], T: float, h: float,
                passes: int, thresh: float) -> Dict[Tuple[int, int], np.ndarray]:
    S = S0
    for _ in range(passes):
        S = relax_pass(S, k, tdist, T, h, thresh)
    return S


def passes_for(k: int) -> int:
    """Number of passes for a family of k sequences (two under 50, else one)."""
    return 2 if k < 50 else 1


def dense_from_csr(row_ptr, col, val, m: int, n: int) -> np.ndarray:
    d = np.zeros((m, n), dtype=np.float64)
    for i in range(m):
        d[i, col[row_ptr[i]:row_ptr[i + 1]]] = val[row_ptr[i]:row_ptr[i + 1]]
    return d
