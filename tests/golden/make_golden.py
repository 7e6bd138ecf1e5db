"""Writes the exact-rational fixtures in this folder.

Calls only ``oracle.bruteforce`` (explicit enumeration of every alignment,
the posterior's definition) in exact rational arithmetic.  Run from the repo
root:  python tests/golden/make_golden.py
"""
import os
import sys
from fractions import Fraction

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import bruteforce as bf  # noqa: E402

ALPHABET = "ARNDCQEGHILKMFPSTWYV"


def joint_table():
    # integer weights w_ab = 1 + ((3a + 7b) mod 11) + 9 [a == b], normalised;
    # deliberately not symmetric
    w = [[1 + ((3 * a + 7 * b) % 11) + (9 if a == b else 0) for b in range(20)] for a in range(20)]
    tot = sum(map(sum, w))
    return w, tot


def main():
    w, tot = joint_table()
    joint = [[Fraction(v, tot) for v in row] for row in w]
    delta = (Fraction(1, 25), Fraction(1, 200))
    eps = (Fraction(1, 2), Fraction(9, 10))
    cases = [("WKDA", "WKA"), ("ACDE", "CADEF"), ("MM", "MMM")]
    with open(os.path.join(HERE, "hmm_exact.txt"), "w") as f:
        f.write("# Exact pair-HMM posteriors by enumeration of every alignment (oracle.bruteforce,\n")
        f.write("# Fraction arithmetic).  Model: pair-HMM of the paper's stage I (Methods, opening\n")
        f.write("# paragraph) with two gap classes, begin/end as match states, no X-Y adjacency.\n")
        f.write("# joint weights w_ab = 1 + ((3a+7b) mod 11) + 9[a==b], p = w / %d\n" % tot)
        f.write("# delta = 1/25 1/200 ; eps = 1/2 9/10\n")
        for xs, ys in cases:
            x = [ALPHABET.index(c) for c in xs]
            y = [ALPHABET.index(c) for c in ys]
            P, Z = bf.hmm_posterior(x, y, joint, delta, eps, exact=True)
            f.write("case %s %s\n" % (xs, ys))
            f.write("Z %s\n" % Z)
            for row in P:
                f.write("row " + " ".join(str(v) for v in row) + "\n")


if __name__ == "__main__":
    main()
