"""Serving loop on the GPU: continuous batching gives each family exactly the
result it gets alone; admission respects the device-memory budget."""
import sys
import time

import numpy as np
import pytest

from paper_1512_07437_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1512_07437_amd import binding
    return binding


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _overlapping(times):
    """Pairs of families whose device work intervals overlapped."""
    iv = sorted((t["launched_s"], t["device_s"]) for t in times)
    return sum(1 for a in range(len(iv)) for b in range(a + 1, len(iv)) if iv[b][0] < iv[a][1])


def _families():
    rng = np.random.default_rng(40)
    fams = []
    for f in range(6):
        k = int(rng.integers(3, 14))
        lens = rng.integers(60, 420, size=k)
        fams.append(W.make_family(k, lens, 1000 + f, r_sub=0.3, r_indel=0.05))
    return fams


KEYS = ("pair_i", "pair_j", "row_off", "row_ptr", "nnz_off", "col", "val", "dist", "log_z")


def test_alone_equals_mix(B, params):
    """Families submitted together run concurrently on the device (their
    device intervals overlap) and each result equals the family run alone,
    bit for bit."""
    p = B.make_params(params)
    rng = np.random.default_rng(41)
    fams = [W.make_family(k, rng.integers(100, 400, size=k), 2000 + f, r_sub=0.3, r_indel=0.05)
            for f, k in enumerate((120, 90, 150, 100, 130, 80))]
    _say("serving: alone")
    alone = [B.qp_posteriors(f, p, 0.01) for f in fams]
    _say("serving: mix")
    srv = B.Server(hbm_budget_bytes=160 << 30, max_slots=4, n_streams=4)
    try:
        tickets = [srv.submit(f, p, 0.01) for f in fams]
        got = [srv.wait(t, timeout_ms=120000) for t in tickets]
    finally:
        srv.close()
    for a, (r, tm) in zip(alone, got):
        for key in KEYS:
            assert np.array_equal(a[key], r[key]), key
        assert tm["submit_s"] <= tm["admit_s"] <= tm["launched_s"] <= tm["device_s"] <= tm["done_s"]
    n_ov = _overlapping([tm for _, tm in got])
    _say("serving: %d overlapping pairs of device intervals" % n_ov)
    assert n_ov >= 1


def test_c4_size_families(B, params):
    """Three families at the top of the C4 size range (k = 500 sequences,
    lengths U{100..600}) served together: each equals its direct run bit for
    bit, and seeded pairs of each match the oracle."""
    import oracle
    p = B.make_params(params)
    fams = []
    for f in range(3):
        rng = np.random.default_rng(4000 + f)
        fams.append(W.make_family(500, rng.integers(100, 601, size=500), 4000 + f, r_sub=0.3, r_indel=0.05))
    srv = B.Server(hbm_budget_bytes=200 << 30, max_slots=3, n_streams=3)
    try:
        tickets = [srv.submit(f, p, 0.01) for f in fams]
        served = [srv.wait(t, timeout_ms=300000) for t in tickets]
    finally:
        srv.close()
    for f, (fam, (res, tm)) in enumerate(zip(fams, served)):
        _say("C4-size family %d: %d pairs, %d entries" % (f, res["n_pairs"], res["nnz"]))
        assert res["n_pairs"] == 500 * 499 // 2 and res["thresh"] == np.float32(0.01)
        direct = B.qp_posteriors(fam, p, 0.01)
        for key in KEYS:
            assert np.array_equal(direct[key], res[key]), (f, key)
        del direct
        rng = np.random.default_rng(44 + f)
        for q in rng.choice(res["n_pairs"], 4, replace=False):
            i, j = W.pair_of_index(int(q), 500)
            orc = oracle.pair(fam[i], fam[j], params, per_model=False)
            rp, col, val = B.pair_csr(res, int(q))
            rows = np.repeat(np.arange(len(fam[i])), np.diff(rp))
            assert np.abs(val.astype(np.float64) - orc["post"][rows, col]).max(initial=0.0) <= 1e-5
            assert abs((1.0 - res["dist"][int(q)]) - orc["ea"]) <= 1e-5


def test_budget_sets_threshold(B, params):
    """Under a budget too small for the output bound at the requested
    threshold, the server admits the family at the smallest larger threshold
    whose bound fits (memory-budgeted sparsity): the result says which, stays
    within that bound, and matches the oracle at that threshold."""
    import oracle
    p = B.make_params(params)
    rng = np.random.default_rng(45)
    fam = W.make_family(8, rng.integers(250, 350, size=8), 45, r_sub=0.3, r_indel=0.05)
    lens = np.array([len(s) for s in fam])
    # the smallest budget (on a 10 % grid) the server takes the family at:
    # what is left for the output there is far below its bound at 0.01
    budget, res = 8 << 20, None
    while res is None:
        srv = B.Server(hbm_budget_bytes=budget, max_slots=1, n_streams=1)
        try:
            t = srv.submit(fam, p, 0.01)
            res = srv.wait(t, timeout_ms=60000)[0]
        except B.QpError as e:
            assert e.status == B.QP_ENOMEM
            budget = int(budget * 1.1)
            assert budget < 4 << 30
        finally:
            srv.close()
    t_used = res["thresh"]
    _say("budget %d bytes: threshold %g" % (budget, t_used))
    assert 0.01 < t_used <= 1.0
    assert res["nnz"] <= B.output_bound(lens, t_used)
    k = 0
    for i in range(8):
        for j in range(i + 1, 8):
            orc = oracle.pair(fam[i], fam[j], params, per_model=False)
            rp, col, val = B.pair_csr(res, k)
            rows = np.repeat(np.arange(len(fam[i])), np.diff(rp))
            assert np.abs(val.astype(np.float64) - orc["post"][rows, col]).max(initial=0.0) <= 1e-5
            g = np.zeros(orc["post"].shape, dtype=bool)
            g[rows, col] = True
            diff = g != (orc["post"] >= t_used)
            assert np.all(np.abs(orc["post"][diff] - t_used) <= 1e-5)
            k += 1


def test_large_family_served_equals_direct(B, params):
    """A family whose outputs span several staging chunks (C2: ~42M entries,
    ~170 MB per array) comes back from the server bit for bit as from
    qp_posteriors."""
    p = B.make_params(params)
    fam = W.c2_family()
    _say("serving: large family direct")
    direct = B.qp_posteriors(fam, p, 0.01)
    _say("serving: large family served")
    srv = B.Server(hbm_budget_bytes=64 << 30, max_slots=2, n_streams=2)
    try:
        res, tm = srv.wait(srv.submit(fam, p, 0.01), timeout_ms=120000)
    finally:
        srv.close()
    assert res["nnz"] > 2 * ((32 << 20) // 4)  # more than two 32 MiB chunks per array
    for key in KEYS:
        assert np.array_equal(direct[key], res[key]), key
    assert tm["admit_s"] <= tm["launched_s"] <= tm["device_s"] <= tm["done_s"]


def test_budget_admission(B, params):
    p = B.make_params(params)
    fams = _families()[:3]
    # a budget too small for any family is rejected at submit
    srv = B.Server(hbm_budget_bytes=1 << 20, max_slots=2, n_streams=2)
    try:
        with pytest.raises(B.QpError) as e:
            srv.submit(fams[0], p, 0.01)
        assert e.value.status == B.QP_ENOMEM
    finally:
        srv.close()
    # one slot: families run one after the other, in arrival order
    _say("serving: one slot")
    srv = B.Server(hbm_budget_bytes=64 << 30, max_slots=1, n_streams=2)
    try:
        ts = [srv.submit(f, p, 0.01) for f in fams]
        times = [srv.wait(t, timeout_ms=60000)[1] for t in ts]
        for a, b in zip(times, times[1:]):
            assert b["admit_s"] >= a["done_s"] - 1e-3
        assert srv.stats()["finished"] == 3
    finally:
        srv.close()


def test_cancel_and_poll(B, params):
    p = B.make_params(params)
    fams = _families()
    srv = B.Server(hbm_budget_bytes=64 << 30, max_slots=1, n_streams=1)
    try:
        ts = [srv.submit(f, p, 0.01) for f in fams[:4]]
        # the last one is still queued behind a single slot
        st = srv.cancel(ts[-1])
        assert st in (B.QP_OK, B.QP_EBUSY)
        with pytest.raises(B.QpError):
            srv.wait(99999, timeout_ms=0)
        for t in ts[:-1]:
            srv.wait(t, timeout_ms=60000)
        if st == B.QP_OK:
            with pytest.raises(B.QpError) as e:
                srv.wait(ts[-1], timeout_ms=1000)
            assert e.value.status == B.QP_ECANCELED
    finally:
        srv.close()


def test_mixed_models_in_one_stream(B, params):
    """Requests carry their own parameters: protein FP32, protein FP64 and
    nucleotide families served side by side each equal their direct run bit
    for bit, and a pair of each meets the oracle at its precision's bar."""
    import oracle
    nt = W.make_nt_params(0)
    jobs = [("protein fp32", _families()[0], params, 0, 1e-5),
            ("protein fp64", _families()[1], params, 1, 1e-7),
            ("nucleotide fp32", W.nt_family(9, [80, 150, 220, 300, 120, 90, 260, 200, 140], 77), nt, 0, 1e-5),
            ("protein fp32 again", _families()[2], params, 0, 1e-5)]
    srv = B.Server(hbm_budget_bytes=32 << 30, max_slots=4, n_streams=4)
    try:
        tickets = [srv.submit(fam, B.make_params(mp, prec), 0.01) for _, fam, mp, prec, _ in jobs]
        served = [srv.wait(t, timeout_ms=120000)[0] for t in tickets]
    finally:
        srv.close()
    for (name, fam, mp, prec, tol), res in zip(jobs, served):
        _say("mixed stream:", name)
        direct = B.qp_posteriors(fam, B.make_params(mp, prec), 0.01)
        for key in KEYS:
            assert np.array_equal(direct[key], res[key]), (name, key)
        orc = oracle.pair(fam[0], fam[1], mp, per_model=False)
        rp, col, val = B.pair_csr(res, 0)
        rows = np.repeat(np.arange(len(fam[0])), np.diff(rp))
        assert np.abs(val.astype(np.float64) - orc["post"][rows, col]).max(initial=0.0) <= tol, name
