"""The C ABI on the CPU: the library loads, exports every function that
include/qp.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1512_07437_amd import workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "qp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qp_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def B():
    from paper_1512_07437_amd import binding
    return binding


def test_every_declared_symbol_is_exported(B):
    names = _declared()
    assert "qp_posteriors" in names and "qp_server_submit" in names
    for name in names:
        assert hasattr(B.lib, name), name
        assert name in B.SIGNATURES, "binding lacks " + name


def test_version(B):
    assert B.qp_version() >> 16 == 1


def test_struct_layout(B):
    # qp_params: 400 doubles, int32 (+pad), 2+2 doubles, 400 doubles, 4 doubles, int32 (+pad)
    assert ctypes.sizeof(B.qp_params) == 8 * 400 + 8 + 8 * 4 + 8 * 400 + 8 * 4 + 8
    assert ctypes.sizeof(B.qp_result) == 4 + 4 + 8 * 3 + 8 * 9 + 8 + 8
    assert ctypes.sizeof(B.qp_request_times) == 8 * 6
    assert ctypes.sizeof(B.qp_tuning) == 4 * 8 + 8 * 9 + 4 * 9 + 4 + 4 + 4  # concurrent_classes, orient, pad to 8
    assert ctypes.sizeof(B.qp_noalloc_out) == 8 * 11
    assert [f[0] for f in B.qp_noalloc_out._fields_ if f[0] != "capacity"] == list(B.NOALLOC_OUT_FIELDS)


def _good(params):
    from paper_1512_07437_amd import binding as B
    return B.make_params(params)


def test_params_check(B, params):
    p = _good(params)
    assert B.qp_params_check(p) == B.QP_OK
    bad = []
    q = _good(params); q.joint[1] += 1e-6; bad.append(q)                 # not symmetric / sum
    q = _good(params); q.n_gap_classes = 3; bad.append(q)
    q = _good(params); q.gap_open[0] = 0.3; q.gap_open[1] = 0.3; bad.append(q)  # tau <= 0
    q = _good(params); q.temperature = 0.0; bad.append(q)
    q = _good(params); q.w_hmm = 1.5; bad.append(q)
    q = _good(params); q.precision = 7; bad.append(q)
    q = _good(params); q.score[3] = float("nan"); bad.append(q)
    q = _good(params); q.gap_extend[0] = 1.0; bad.append(q)
    for q in bad:
        assert B.qp_params_check(q) == B.QP_EINVAL
        assert B.qp_last_error()


def test_validation_before_device(B, params):
    p = _good(params)
    fam = W.c1_family()[:3]
    with pytest.raises(B.QpError) as e:
        B.qp_posteriors(fam[:2] + [np.zeros(0, np.uint8)], p, 0.01)
    assert e.value.status == B.QP_EINVAL and "lens[2]" in str(e.value)
    bad = fam[0].copy()
    bad[5] = 20
    with pytest.raises(B.QpError) as e:
        B.qp_posteriors([bad, fam[1]], p, 0.01)
    assert e.value.status == B.QP_EINVAL and "residue" in str(e.value)
    for t in (0.0, -1.0, 1.5, float("nan")):
        with pytest.raises(B.QpError) as e:
            B.qp_posteriors(fam, p, t)
        assert e.value.status == B.QP_EINVAL
    with pytest.raises(B.QpError) as e:
        B.qp_posteriors_pairs(fam, [0], [0], p, 0.01)
    assert e.value.status == B.QP_EINVAL
    with pytest.raises(B.QpError) as e:
        B.qp_posteriors_pairs(fam, [0], [3], p, 0.01)
    assert e.value.status == B.QP_EINVAL


def test_long_sequences_refused(B, params):
    """Sequences longer than QP_MAX_SEQ_LEN (1536) are refused before any
    device call; exactly the limit passes validation (it then needs a GPU)."""
    p = _good(params)
    rng = np.random.default_rng(7)
    long_seq = rng.integers(0, 20, size=1537).astype(np.uint8)
    short = rng.integers(0, 20, size=50).astype(np.uint8)
    with pytest.raises(B.QpError) as e:
        B.qp_posteriors([short, long_seq], p, 0.01)
    assert e.value.status == B.QP_EINVAL and "1537 > 1536" in str(e.value)
    with pytest.raises(B.QpError) as e:
        B.Plan([50, 1537], p, 0.01)
    assert e.value.status == B.QP_EINVAL


def test_empty_family_needs_no_device(B, params):
    p = _good(params)
    for fam in ([], W.c1_family()[:1]):
        r = B.qp_posteriors(fam, p, 0.01)
        assert r["n_pairs"] == 0 and r["nnz"] == 0
        assert list(r["row_off"]) == [0] and list(r["nnz_off"]) == [0]
    r = B.qp_posteriors_pairs(W.c1_family(), [], [], p, 0.01)
    assert r["n_pairs"] == 0


def _hip_devices() -> int:
    try:
        hip = ctypes.CDLL("libamdhip64.so")
    except OSError:
        return 0
    n = ctypes.c_int(0)
    return n.value if hip.hipGetDeviceCount(ctypes.byref(n)) == 0 else 0


def test_no_device_is_reported(B, params):
    if _hip_devices() > 0:
        pytest.skip("a GPU is present")
    with pytest.raises(B.QpError) as e:
        B.qp_posteriors(W.c1_family()[:2], _good(params), 0.01)
    assert e.value.status == B.QP_EDEVICE


def test_result_free_null_safe(B):
    B.lib.qp_result_free(None)
    B.lib.qp_plan_destroy(None)


def test_server_config_errors(B):
    for cfg in [(0, 4, 2), (1 << 30, 0, 2), (1 << 30, 65, 2), (1 << 30, 4, 0), (1 << 30, 4, 17)]:
        with pytest.raises(B.QpError) as e:
            B.Server(*cfg)
        assert e.value.status in (B.QP_EINVAL, B.QP_EDEVICE)


def test_tuning_table(B):
    """qp_set_tuning / qp_get_tuning: values round-trip, out-of-range values
    are refused and leave the table unchanged, NULL restores the default."""
    before = B.get_tuning()
    try:
        B.set_tuning([2, 3, 3, 5, 6, 7, 8, 8], [1.0, 0.5, 0.75, 1.0, 1.0, 1.0, 1.0, 1.0, 0.25])
        t = B.get_tuning()
        assert t["rows_per_lane"] == [2, 3, 3, 5, 6, 7, 8, 8]
        assert t["waves_frac"] == [1.0, 0.5, 0.75, 1.0, 1.0, 1.0, 1.0, 1.0, 0.25]
        for bad_r, bad_w in (([0, 2, 3, 4, 5, 6, 7, 8], None),   # fewer rows per lane than the bucket needs
                             ([1, 1, 3, 4, 5, 6, 7, 8], None),
                             ([1, 2, 3, 4, 5, 6, 7, 9], None),   # more than 8
                             (None, [0.0] + [1.0] * 8),
                             (None, [1.0] * 8 + [1.5])):
            with pytest.raises(B.QpError) as e:
                B.set_tuning(bad_r, bad_w)
            assert e.value.status == B.QP_EINVAL
            assert B.get_tuning() == t
        B.set_tuning(recompute=[1, 0, 1, 1, 0, 0, 0, 0, 0])
        assert B.get_tuning()["recompute"] == [1, 0, 1, 1, 0, 0, 0, 0, 0]
        t = B.get_tuning()
        for bad in ([2] + [0] * 8, [0] * 5 + [1] + [0] * 3, [0] * 7 + [1, 0]):
            with pytest.raises(B.QpError) as e:
                B.set_tuning(recompute=bad)
            assert e.value.status == B.QP_EINVAL and B.get_tuning() == t
        B.set_tuning()
        d = B.get_tuning()
        assert d["rows_per_lane"] == list(range(1, 9)) and d["waves_frac"] == [1.0] * 9
        assert d["recompute"] == [1, 1, 1, 1, 1, 0, 0, 0, 0] and d["concurrent_classes"] == 1 and d["orient"] == 1
        B.set_tuning(concurrent_classes=0)
        assert B.get_tuning()["concurrent_classes"] == 0
        t = B.get_tuning()
        with pytest.raises(B.QpError) as e:
            B.set_tuning(concurrent_classes=2)
        assert e.value.status == B.QP_EINVAL and B.get_tuning() == t
        B.set_tuning(orient=0)
        assert B.get_tuning()["orient"] == 0
        t = B.get_tuning()
        with pytest.raises(B.QpError) as e:
            B.set_tuning(orient=3)
        assert e.value.status == B.QP_EINVAL and B.get_tuning() == t
    finally:
        B.set_tuning(before["rows_per_lane"], before["waves_frac"], before["recompute"],
                     before["concurrent_classes"], before["orient"])


def test_tuning_file_is_valid(B):
    """The committed autotuned table, if present, is accepted by the library."""
    import json
    if not os.path.exists(B.TUNING_PATH):
        pytest.skip("no tuning table measured yet")
    d = json.load(open(B.TUNING_PATH))
    t = B.qp_tuning()
    t.rows_per_lane[:] = d["rows_per_lane"]
    t.waves_frac[:] = d["waves_frac"]
    assert B.lib.qp_set_tuning(ctypes.byref(t)) == 0
    assert B.get_tuning()["rows_per_lane"] == d["rows_per_lane"]


def test_noalloc_validation_before_device(B, params):
    """The allocation-free entry point checks its inputs, and that the
    caller's output capacity covers the output bound, before any device call."""
    p = _good(params)
    lens = [50, 60, 70]
    ptrs = {k: 4096 for k in B.NOALLOC_OUT_FIELDS}
    bound = B.output_bound(lens, 0.01)
    with pytest.raises(B.QpError) as e:
        B.posteriors_noalloc(4096, 4096, lens, p, 0.01, ptrs, bound - 1, 0)
    assert e.value.status == B.QP_EINVAL and "output bound" in str(e.value)
    with pytest.raises(B.QpError) as e:
        B.posteriors_noalloc(4096, 4096, [50, 0], p, 0.01, ptrs, bound, 0)
    assert e.value.status == B.QP_EINVAL
    with pytest.raises(B.QpError) as e:
        B.posteriors_noalloc(4096, 4096, lens, p, 1.5, ptrs, bound, 0)
    assert e.value.status == B.QP_EINVAL
    missing = dict(ptrs, col=0)
    with pytest.raises(B.QpError) as e:
        B.posteriors_noalloc(4096, 4096, lens, p, 0.01, missing, bound, 0)
    assert e.value.status == B.QP_EINVAL
    if _hip_devices() == 0:
        with pytest.raises(B.QpError) as e:
            B.posteriors_noalloc(4096, 4096, lens, p, 0.01, ptrs, bound, 0)
        assert e.value.status == B.QP_EDEVICE


def test_relax_validation_before_device(B):
    """qp_relax_create checks its arguments before any device call."""
    lens = [50, 60, 70]
    for args in ((-1, 3.0, 1, 0.01), (200, 0.5, 1, 0.01), (200, 3.0, 0, 0.01), (200, 3.0, 9, 0.01),
                 (200, 3.0, 1, 0.0), (200, float("nan"), 1, 0.01)):
        with pytest.raises(B.QpError) as e:
            B.Relax(lens, *args)
        assert e.value.status == B.QP_EINVAL
    with pytest.raises(B.QpError) as e:
        B.Relax([50, 0], 200, 3.0, 1, 0.01)
    assert e.value.status == B.QP_EINVAL
    with pytest.raises(B.QpError) as e:
        B.Relax([50] * 2049, 200, 3.0, 1, 0.01)
    assert e.value.status == B.QP_EINVAL and "2048" in str(e.value)
