"""Seeded synthetic protein families and model parameters.

This module is the one piece of code that both the HIP path and the CPU
oracle consume.  It produces *inputs* only -- residue codes, the raw model
parameters (a joint emission matrix, gap probabilities, an integer score
matrix, PF gap scores, temperature) and the family shapes -- and performs none
of the posterior arithmetic.  Each side derives its own tables from the raw
parameters.

The paper's benchmarks (BAliBASE, BaliFam, HomFam; Methods, "Accuracy
assessment") are not available, and their items are not reproduced.  The
families here borrow only their shape: a few to a thousand sequences of
protein-like length, evolved from a common root.

Residue alphabet: 20 amino-acid codes 0..19 in the order ``ARNDCQEGHILKMFPSTWYV``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

ALPHABET = "ARNDCQEGHILKMFPSTWYV"
K = 20


# --------------------------------------------------------------------------
# model parameters
# --------------------------------------------------------------------------
@dataclasses.dataclass
class ModelParams:
    """Raw parameters of the two posterior models (pair-HMM and partition
    function).  Field names mirror ``qp_params`` in ``include/qp.h``."""

    joint: np.ndarray            # [20,20] symmetric joint emission p_ab, sums to 1
    gap_open: Tuple[float, ...]  # delta_k per gap class (HMM)
    gap_extend: Tuple[float, ...]  # epsilon_k per gap class (HMM)
    score: np.ndarray            # [20,20] symmetric PF substitution scores
    pf_gap_open: float           # PF score of the first residue of a gap run
    pf_gap_extend: float         # PF score of each further residue of a run
    temperature: float           # PF temperature T
    w_hmm: float = 0.5           # P = w*P_hmm + (1-w)*P_pf
    alphabet: int = 20           # residue codes 0..alphabet-1 (4: nucleotides)

    @property
    def n_gap_classes(self) -> int:
        return len(self.gap_open)

    def copy(self, **kw) -> "ModelParams":
        d = dataclasses.asdict(self)
        d.update(kw)
        d["joint"] = np.array(d["joint"], dtype=np.float64)
        d["score"] = np.array(d["score"], dtype=np.float64)
        return ModelParams(**d)


def make_params(seed: int = 0, *, gap_open=(0.02, 0.005), gap_extend=(0.5, 0.9),
                pf_gap_open=-12.0, pf_gap_extend=-1.0, temperature=5.0,
                w_hmm=0.5) -> ModelParams:
    """Seeded symmetric joint emission and the derived integer score matrix.

    joint: A_ab ~ U(0,1) i.i.d., J = (A + A^T)/2 + 4 I, p = J / sum(J).
    score: s_ab = round(2 * log2(p_ab / (q_a q_b))) with q the row sums of p
    (half-bit units, the usual convention for protein score matrices).  The
    score matrix is an *input* to the partition function; the HMM and the PF
    sides each rebuild their own weights from these raw numbers.
    """
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 1.0, size=(K, K))
    j = (a + a.T) / 2.0 + 4.0 * np.eye(K)
    p = j / j.sum()
    q = p.sum(axis=1)
    score = np.round(2.0 * np.log2(p / np.outer(q, q)))
    return ModelParams(joint=p, gap_open=tuple(gap_open), gap_extend=tuple(gap_extend),
                       score=score.astype(np.float64), pf_gap_open=float(pf_gap_open),
                       pf_gap_extend=float(pf_gap_extend), temperature=float(temperature),
                       w_hmm=float(w_hmm))


def background(params: ModelParams) -> np.ndarray:
    """Residue background used to draw roots and inserted residues: the
    marginal of the seeded joint emission (self-consistent stand-in for the
    standard amino-acid frequencies, which are not reproduced here)."""
    q = params.joint.sum(axis=1)
    return q / q.sum()


def substitution_matrix(seed: int = 0) -> np.ndarray:
    """Row-stochastic 20x20 substitution kernel with zero diagonal.  Drawn from
    the same generator as the joint emission, after it: row a ~ Dirichlet(1)
    over the 19 other residues."""
    rng = np.random.default_rng(seed)
    rng.uniform(0.0, 1.0, size=(K, K))  # advance past the joint draw
    r = np.zeros((K, K))
    for a in range(K):
        w = rng.dirichlet(np.ones(K - 1))
        r[a, [b for b in range(K) if b != a]] = w
    return r


# --------------------------------------------------------------------------
# evolution model
# --------------------------------------------------------------------------
def evolve(root: np.ndarray, rng: np.random.Generator, q: np.ndarray, subst: np.ndarray,
           r_sub: float, r_indel: float) -> np.ndarray:
    """One leaf of a star tree.  Per root site: substitute with probability
    ``r_sub`` (new residue from the substitution row), then with probability
    ``r_indel`` open an indel after it: half the time delete the following run
    of sites, otherwise insert a run of background residues; run lengths are
    geometric with mean 3.  Deleted sites are skipped together with any indel
    they would have opened."""
    L = len(root)
    root = np.asarray(root, dtype=np.int64)
    # substitutions (inverse-CDF draw from the row of the old residue)
    cdf = np.cumsum(subst, axis=1)
    tot = cdf[:, -1:]
    cdf = np.divide(cdf, tot, out=np.zeros_like(cdf), where=tot > 0)  # rows of absent letters stay 0
    sub = rng.random(L) < r_sub
    u = rng.random(L)
    new = (cdf[root] > u[:, None]).argmax(axis=1)
    site = np.where(sub, new, root)
    # indel events after each site
    ev = rng.random(L) < r_indel
    kind_del = rng.random(L) < 0.5
    glen = rng.geometric(1.0 / 3.0, size=L)
    # residues of every potential insertion, drawn at once (inverse CDF of q)
    ins_len = np.where(ev & ~kind_del, glen, 0)
    ins_end = np.cumsum(ins_len)
    qc = np.cumsum(q)
    qc /= qc[-1]
    pool = np.minimum(np.searchsorted(qc, rng.random(int(ins_end[-1]) if L else 0), side="right"), K - 1)
    out: List[np.ndarray] = []
    i = 0
    for e in np.flatnonzero(ev):
        if e < i:
            continue  # inside a deletion
        out.append(site[i:e + 1])
        if kind_del[e]:
            i = e + 1 + int(glen[e])
        else:
            out.append(pool[ins_end[e] - ins_len[e]: ins_end[e]])
            i = e + 1
    if i < L:
        out.append(site[i:])
    return (np.concatenate(out) if out else np.zeros(0, np.int64)).astype(np.uint8)


def fit_length(seq: np.ndarray, target: int, rng: np.random.Generator, q: np.ndarray) -> np.ndarray:
    """Random contiguous window if the leaf is too long; i.i.d. background
    residues appended if it is too short."""
    if len(seq) >= target:
        off = int(rng.integers(0, len(seq) - target + 1))
        return np.ascontiguousarray(seq[off:off + target])
    extra = rng.choice(K, size=target - len(seq), p=q).astype(np.uint8)
    return np.concatenate([seq, extra]).astype(np.uint8)


def make_family(n: int, lengths: Sequence[int], seed, *, r_sub: float = 0.3,
                r_indel: float = 0.05, params: Optional[ModelParams] = None,
                root_len: Optional[int] = None, subst: Optional[np.ndarray] = None) -> List[np.ndarray]:
    """A family of ``n`` sequences with the given target lengths, all evolved
    from one random root of length ``root_len`` (default: the longest target)."""
    params = params or make_params(0)
    q = background(params)
    subst = substitution_matrix(0) if subst is None else subst
    rng = np.random.default_rng(seed)
    root_len = int(root_len or max(lengths))
    root = rng.choice(K, size=root_len, p=q).astype(np.uint8)
    fam = []
    for t in range(n):
        leaf = evolve(root, rng, q, subst, r_sub, r_indel)
        fam.append(fit_length(leaf, int(lengths[t]), rng, q))
    return fam


# --------------------------------------------------------------------------
# nucleotide mode
# --------------------------------------------------------------------------
NT_ALPHABET = "ACGT"


def make_nt_params(seed: int = 0, **kw) -> ModelParams:
    """Nucleotide model (codes 0..3 = ACGT).  The nucleotide tables the
    method names are not available; this stand-in applies the protein recipe
    to four letters: A_ab ~ U(0,1), J = (A + A^T)/2 + 4 I, p = J / sum(J),
    s_ab = round(2 log2(p_ab / (q_a q_b))), embedded in the 20 x 20 layout
    with zeros outside the 4 x 4 block.  Gap and PF settings as for proteins
    unless given."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 1.0, size=(4, 4))
    j = (a + a.T) / 2.0 + 4.0 * np.eye(4)
    p4 = j / j.sum()
    q4 = p4.sum(axis=1)
    joint = np.zeros((K, K))
    joint[:4, :4] = p4
    score = np.zeros((K, K))
    score[:4, :4] = np.round(2.0 * np.log2(p4 / np.outer(q4, q4)))
    d = dict(gap_open=(0.02, 0.005), gap_extend=(0.5, 0.9), pf_gap_open=-12.0, pf_gap_extend=-1.0,
             temperature=5.0, w_hmm=0.5)
    d.update(kw)
    return ModelParams(joint=joint, gap_open=tuple(d["gap_open"]), gap_extend=tuple(d["gap_extend"]), score=score,
                       pf_gap_open=float(d["pf_gap_open"]), pf_gap_extend=float(d["pf_gap_extend"]),
                       temperature=float(d["temperature"]), w_hmm=float(d["w_hmm"]), alphabet=4)


def nt_substitution_matrix(seed: int = 0) -> np.ndarray:
    """Row-stochastic 4 x 4 substitution kernel with zero diagonal (rows
    Dirichlet(1) over the three other letters), in the 20 x 20 layout."""
    rng = np.random.default_rng(seed)
    rng.uniform(0.0, 1.0, size=(4, 4))  # advance past the joint draw
    r = np.zeros((K, K))
    for a in range(4):
        r[a, [b for b in range(4) if b != a]] = rng.dirichlet(np.ones(3))
    return r


def nt_family(n: int, lengths: Sequence[int], seed, *, r_sub: float = 0.3, r_indel: float = 0.05) -> List[np.ndarray]:
    """Nucleotide family: the evolution model of the protein families over
    the four letters of the nucleotide model."""
    return make_family(n, lengths, seed, r_sub=r_sub, r_indel=r_indel, params=make_nt_params(0),
                       subst=nt_substitution_matrix(0))


def nt_workload_family() -> List[np.ndarray]:
    """200 nucleotide sequences, lengths U{250..350}, seed 6 (the C2 shape)."""
    rng = np.random.default_rng(6)
    lens = rng.integers(250, 351, size=200)
    return nt_family(200, lens, np.random.SeedSequence(6))


# --------------------------------------------------------------------------
# the five workload shapes
# --------------------------------------------------------------------------
def c1_family() -> List[np.ndarray]:
    """8 sequences, lengths U{80..120}, substitution 0.3, indel 0.05, seed 1."""
    rng = np.random.default_rng(1)
    lens = rng.integers(80, 121, size=8)
    return make_family(8, lens, np.random.SeedSequence(1), r_sub=0.3, r_indel=0.05)


def c2_family() -> List[np.ndarray]:
    """200 sequences, lengths U{250..350}, seed 2 (19,900 pairs)."""
    rng = np.random.default_rng(2)
    lens = rng.integers(250, 351, size=200)
    return make_family(200, lens, np.random.SeedSequence(2), r_sub=0.3, r_indel=0.05)


def c2_sample() -> np.ndarray:
    """Seeded 200-pair sample of C2's 19,900 pair indices."""
    return np.sort(np.random.default_rng(22).choice(19900, 200, replace=False))


def c3_family() -> List[np.ndarray]:
    """1,000 sequences, lengths round(exp(U(ln 50, ln 1500))), seed 3."""
    rng = np.random.default_rng(3)
    lens = np.round(np.exp(rng.uniform(math.log(50), math.log(1500), size=1000))).astype(int)
    return make_family(1000, lens, np.random.SeedSequence(3), r_sub=0.3, r_indel=0.05)


def c3_sample(lens: Sequence[int], parts: bool = False):
    """200-pair sample of C3: 150 uniform + 50 from the top 1% by m*n (with
    ``parts``, the two sorted parts separately)."""
    n = len(lens)
    P = n * (n - 1) // 2
    rng = np.random.default_rng(33)
    ii, jj = np.triu_indices(n, 1)
    cost = np.asarray(lens)[ii].astype(np.int64) * np.asarray(lens)[jj]
    top = np.argsort(-cost, kind="stable")[: max(1, P // 100)]
    uni = rng.choice(P, 150, replace=False)
    rest = np.setdiff1d(top, uni)
    big = rng.choice(rest, 50, replace=False)
    if parts:
        return np.sort(uni), np.sort(big)
    return np.sort(np.concatenate([uni, big]))


def c4_stream(n_families: int = 2000, seed: int = 4, rate: float = 20.0):
    """Poisson stream of families: exponential inter-arrivals (mean 1/rate,
    50 ms by default), sizes U{10..500}, lengths U{100..600}, each family
    from its own root.  Yields (arrival_seconds, family)."""
    ss = np.random.SeedSequence(seed)
    rng = np.random.default_rng(ss)
    children = ss.spawn(n_families)
    t = 0.0
    for f in range(n_families):
        t += float(rng.exponential(1.0 / rate))
        frng = np.random.default_rng(children[f])
        k = int(frng.integers(10, 501))
        lens = frng.integers(100, 601, size=k)
        fam = make_family(k, lens, children[f], r_sub=0.3, r_indel=0.05)
        yield t, fam


def c5_pairs(n_pairs: int = 64, seed: int = 5, lo: int = 3000, hi: int = 5000) -> List[Tuple[np.ndarray, np.ndarray]]:
    """64 independent divergent pairs, each from its own root, lengths
    U{lo..hi} (default 3000..5000), substitution 0.6, indel 0.1."""
    ss = np.random.SeedSequence(seed)
    out = []
    for child in ss.spawn(n_pairs):
        rng = np.random.default_rng(child)
        lens = rng.integers(lo, hi + 1, size=2)
        a, b = make_family(2, lens, child, r_sub=0.6, r_indel=0.1)
        out.append((a, b))
    return out


def c5p_pairs(n_pairs: int = 64, seed: int = 55, lo: int = 1000, hi: int = 1536,
              r_sub: float = 0.3, r_indel: float = 0.05) -> List[Tuple[np.ndarray, np.ndarray]]:
    """Precision workload within the supported lengths: 64 independent pairs,
    each from its own root, lengths U{1000..1536} (up to three 512-row
    bands), with the substitution and indel rates of the other workloads."""
    ss = np.random.SeedSequence(seed)
    out = []
    for child in ss.spawn(n_pairs):
        rng = np.random.default_rng(child)
        lens = rng.integers(lo, hi + 1, size=2)
        a, b = make_family(2, lens, child, r_sub=r_sub, r_indel=r_indel)
        out.append((a, b))
    return out


def pair_index(i: int, j: int, n: int) -> int:
    """Row-major index of pair (i<j) among the n(n-1)/2 pairs of a family."""
    return i * n - i * (i + 1) // 2 + (j - i - 1)


def pair_of_index(p: int, n: int) -> Tuple[int, int]:
    i = 0
    while p >= n - 1 - i:
        p -= n - 1 - i
        i += 1
    return i, i + 1 + p


def random_family(rng: np.random.Generator, n: int, lo: int, hi: int) -> List[np.ndarray]:
    """Unrelated i.i.d. uniform sequences (edge-case tests)."""
    return [rng.integers(0, K, size=int(rng.integers(lo, hi + 1))).astype(np.uint8) for _ in range(n)]


def encode(s: str) -> np.ndarray:
    return np.asarray([ALPHABET.index(c) for c in s], dtype=np.uint8)


def decode(a: np.ndarray) -> str:
    return "".join(ALPHABET[int(c)] for c in a)
