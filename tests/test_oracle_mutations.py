"""The pins must catch plausible mistakes in the oracle.

Each case copies ``oracle/qp_oracle.c`` to a temporary directory, plants one
mistake (a dropped term, a wrong coefficient or sign, a transposed operand, a
wrong marginal, ...), builds it with gcc and checks that the brute-force pins
reject the mutant.  The committed oracle is never modified.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import bruteforce as bf
from paper_1512_07437_amd import workload as W

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "qp_oracle.c")

MUTANTS = {
    "drop_Y_into_M": ("into = lse2(into, md->l_close[k] + FY(k, i - 1, j - 1));", ""),
    "X_extend_uses_open": ("md->l_ext[k] + FX(k, i - 1, j))", "md->l_open[k] + FX(k, i - 1, j))"),
    "transposed_emission": ("x[(i) - 1] * QPO_ALPHA + y[(j) - 1]", "y[(j) - 1] * QPO_ALPHA + x[(i) - 1]"),
    "close_sign": ("md->l_close[k] = log(1.0 - eps[k]);", "md->l_close[k] = log(1.0 + eps[k]);"),
    "tau_single_delta": ("tau -= 2.0 * delta[k];", "tau -= delta[k];"),
    "bwd_Y_open_as_ext": ("vm = lse2(vm, md->l_open[k] + BY(k, i, j + 1));",
                          "vm = lse2(vm, md->l_ext[k] + BY(k, i, j + 1));"),
    "mea_no_up": ("if (up > v) v = up;", ""),
    "combination_weight": ("w_hmm * ph[c] + (1.0 - w_hmm) * pp[c]", "w_hmm * ph[c] + w_hmm * pp[c]"),
    "y_marginal_from_rows": ("qy[c] += joint[a * QPO_ALPHA + c];", "qy[c] += joint[c * QPO_ALPHA + a];"),
    "pf_extend_is_open": ("md->l_ext[0] = g_ext / T;", "md->l_ext[0] = g_open / T;"),
    "end_not_match": ("if (i == m && j == n) t = 0.0;", "if (i == m && j == n) t = md->l_mm;"),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert old in src, "mutation anchor not found: " + name
    mutated = src.replace(old, new, 1)
    c = tmp_path / (name + ".c")
    so = tmp_path / (name + ".so")
    c.write_text(mutated)
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-std=c99", "-o", str(so), str(c), "-lm"])
    lib = ctypes.CDLL(str(so))
    d = ctypes.POINTER(ctypes.c_double)
    u8 = ctypes.POINTER(ctypes.c_uint8)
    lib.qpo_pair.argtypes = [u8, ctypes.c_int, u8, ctypes.c_int, d, ctypes.c_int, d, d, d,
                             ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, d, d, d, d]
    return lib


def _run(lib, x, y, p):
    m, n = len(x), len(y)
    f = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    joint, score, delta, eps = f(p.joint), f(p.score), f(p.gap_open), f(p.gap_extend)
    post, ph, pp, st = np.zeros((m, n)), np.zeros((m, n)), np.zeros((m, n)), np.zeros(6)
    D = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    U = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    lib.qpo_pair(U(x), m, U(y), n, D(joint), len(delta), D(delta), D(eps), D(score), p.pf_gap_open,
                 p.pf_gap_extend, p.temperature, p.w_hmm, D(post), D(ph), D(pp), D(st))
    return post, ph, pp, st


def _pins_pass(lib) -> bool:
    rng = np.random.default_rng(2024)
    for (m, n) in [(2, 3), (4, 3), (3, 5), (5, 5)]:
        A = rng.uniform(0.05, 1.0, size=(20, 20))
        p = W.ModelParams(joint=A / A.sum(), gap_open=(0.05, 0.01), gap_extend=(0.4, 0.85),
                          score=rng.normal(0, 3, size=(20, 20)), pf_gap_open=-4.0, pf_gap_extend=-1.5,
                          temperature=2.5, w_hmm=0.35)
        x = rng.integers(0, 20, m).astype(np.uint8)
        y = rng.integers(0, 20, n).astype(np.uint8)
        post, ph, pp, st = _run(lib, x, y, p)
        Ph, Zh = bf.hmm_posterior(x, y, p.joint, p.gap_open, p.gap_extend)
        Pp, lZp = bf.pf_posterior(x, y, p.score, p.pf_gap_open, p.pf_gap_extend, p.temperature)
        comb = p.w_hmm * np.array(Ph) + (1 - p.w_hmm) * np.array(Pp)
        ok = (np.allclose(ph, Ph, rtol=0, atol=1e-12) and np.allclose(pp, Pp, rtol=0, atol=1e-12)
              and abs(st[0] - np.log(Zh)) < 1e-10 and abs(st[2] - lZp) < 1e-10
              and abs(st[0] - st[1]) < 1e-10 and abs(st[2] - st[3]) < 1e-10
              and np.allclose(post, comb, rtol=0, atol=1e-12)
              and abs(st[4] - bf.mea_brute(comb)) < 1e-12)
        if not ok:
            return False
    return True


def test_unmutated_copy_passes(tmp_path):
    assert _pins_pass(_build(tmp_path, "identity", "#include <math.h>", "#include <math.h>"))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    assert not _pins_pass(_build(tmp_path, name, old, new))
