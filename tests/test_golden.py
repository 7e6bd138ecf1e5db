"""The FP64 oracle against the exact-rational fixtures in tests/golden/
(written by tests/golden/make_golden.py from explicit enumeration)."""
import math
import os
from fractions import Fraction

import numpy as np

import oracle
from paper_1512_07437_amd import workload as W

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hmm_exact.txt")


def _cases():
    cases, cur = [], None
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        tag, rest = line.split(" ", 1)
        if tag == "case":
            cur = dict(xy=rest.split(), rows=[])
            cases.append(cur)
        elif tag == "Z":
            cur["Z"] = Fraction(rest.strip())
        elif tag == "row":
            cur["rows"].append([Fraction(v) for v in rest.split()])
    return cases


def test_oracle_matches_exact_fixture():
    w = np.array([[1 + ((3 * a + 7 * b) % 11) + (9 if a == b else 0) for b in range(20)] for a in range(20)],
                 dtype=np.float64)
    p = W.ModelParams(joint=w / w.sum(), gap_open=(1 / 25, 1 / 200), gap_extend=(0.5, 0.9),
                      score=np.zeros((20, 20)), pf_gap_open=-1.0, pf_gap_extend=-1.0, temperature=1.0)
    cases = _cases()
    assert len(cases) == 3
    for c in cases:
        x, y = W.encode(c["xy"][0]), W.encode(c["xy"][1])
        r = oracle.pair(x, y, p)
        exact = np.array([[float(v) for v in row] for row in c["rows"]])
        np.testing.assert_allclose(r["post_h"], exact, rtol=0, atol=1e-13)
        assert abs(r["logz_h"] - math.log(float(c["Z"]))) < 1e-12
