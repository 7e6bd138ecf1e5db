"""Nucleotide mode (alphabet 4): parameters, validation and the oracle on the
four-letter model, on the CPU.  The joint emission keeps the 20 x 20 layout
with zeros outside the 4 x 4 block; every posterior is defined by the same
recurrences, so the oracle is pinned against enumeration exactly as for
proteins."""
import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf
from paper_1512_07437_amd import workload as W

# letters outside the alphabet have zero marginals: their emission entries are
# 0/0 in the floating-point enumeration and never read
pytestmark = pytest.mark.filterwarnings("ignore:invalid value encountered in divide:RuntimeWarning")


@pytest.fixture(scope="module")
def B():
    from paper_1512_07437_amd import binding
    return binding


def test_nt_params_and_family():
    mp = W.make_nt_params(0)
    assert mp.alphabet == 4
    assert abs(mp.joint.sum() - 1.0) < 1e-12 and np.allclose(mp.joint, mp.joint.T)
    assert np.all(mp.joint[4:, :] == 0) and np.all(mp.joint[:, 4:] == 0) and np.all(mp.joint[:4, :4] > 0)
    fam = W.nt_family(6, [40, 50, 60, 70, 80, 90], 2)
    assert [len(s) for s in fam] == [40, 50, 60, 70, 80, 90]
    assert max(int(s.max()) for s in fam) <= 3
    assert W.nt_family(3, [30, 30, 30], 5)[1].tolist() == W.nt_family(3, [30, 30, 30], 5)[1].tolist()


def test_params_check_alphabet(B):
    p = B.make_params(W.make_nt_params(0))
    assert p.alphabet == 4 and B.qp_params_check(p) == B.QP_OK
    p.joint[4 * 20 + 4] = 1e-3  # mass outside the alphabet
    assert B.qp_params_check(p) == B.QP_EINVAL
    for a in (1, 21, -3):
        q = B.make_params(W.make_nt_params(0))
        q.alphabet = a
        assert B.qp_params_check(q) == B.QP_EINVAL
    prot = B.make_params(W.make_params(0))
    assert prot.alphabet == 20 and B.qp_params_check(prot) == B.QP_OK
    prot.alphabet = 0  # reads as 20
    assert B.qp_params_check(prot) == B.QP_OK


def test_codes_outside_alphabet_refused_before_device(B):
    p = B.make_params(W.make_nt_params(0))
    seqs = [np.array([0, 1, 2, 3], np.uint8), np.array([0, 4, 1], np.uint8)]
    with pytest.raises(B.QpError) as e:
        B.qp_posteriors(seqs, p, 0.01)
    assert e.value.status == B.QP_EINVAL and "residue code" in str(e.value)


@pytest.mark.parametrize("seed", range(8))
def test_oracle_equals_enumeration_nt(seed):
    """Both models and their average on four-letter pairs of up to 6 x 6
    residues: the oracle's DP against every alignment, one by one."""
    rng = np.random.default_rng(40 + seed)
    mp = W.make_nt_params(int(rng.integers(0, 5)), temperature=float(rng.uniform(1, 6)))
    m, n = int(rng.integers(1, 7)), int(rng.integers(1, 7))
    x = rng.integers(0, 4, m).astype(np.uint8)
    y = rng.integers(0, 4, n).astype(np.uint8)
    r = oracle.pair(x, y, mp)
    Ph, _ = bf.hmm_posterior(x, y, mp.joint, mp.gap_open, mp.gap_extend)
    Pp, _ = bf.pf_posterior(x, y, mp.score, mp.pf_gap_open, mp.pf_gap_extend, mp.temperature)
    comb = mp.w_hmm * np.array(Ph) + (1 - mp.w_hmm) * np.array(Pp)
    assert np.all(np.isfinite(r["post"]))
    np.testing.assert_allclose(r["post"], comb, rtol=0, atol=1e-12)
    assert abs(r["mea"] - bf.mea_brute(comb)) < 1e-12
