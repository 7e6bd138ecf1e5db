"""The allocation-free entry point (qp_posteriors_noalloc) against the plan
form it is a variant of (qp_plan_create with the output sized to the bound,
then qp_plan_run): two calls in a row, the second on a smaller family, each
equal to the plan's outputs, with no device memory taken by the second call."""
import numpy as np
import pytest

from paper_1512_07437_amd import workload as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[no-alloc]", *a, flush=True)


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.zeros(1, device="cuda:0")  # torch's runtime first
    from paper_1512_07437_amd import binding
    return binding


def _outputs(torch, lens, thresh, B):
    n = len(lens)
    P = n * (n - 1) // 2
    rows = sum(int(lens[i]) + 1 for i in range(n) for _ in range(i + 1, n))
    cap = B.output_bound(lens, thresh)
    dev = "cuda:0"
    t = dict(pair_i=torch.full((max(P, 1),), -1, dtype=torch.int32, device=dev),
             pair_j=torch.full((max(P, 1),), -1, dtype=torch.int32, device=dev),
             row_off=torch.full((P + 1,), -1, dtype=torch.int64, device=dev),
             row_ptr=torch.full((max(rows, 1),), -1, dtype=torch.int32, device=dev),
             nnz_off=torch.full((P + 1,), -1, dtype=torch.int64, device=dev),
             col=torch.full((cap,), -1, dtype=torch.int32, device=dev),
             val=torch.full((cap,), -1.0, dtype=torch.float32, device=dev),
             dist=torch.full((max(P, 1),), -1.0, dtype=torch.float64, device=dev),
             log_z=torch.full((max(2 * P, 1),), -1.0, dtype=torch.float64, device=dev),
             status=torch.full((1,), -1, dtype=torch.int32, device=dev))
    return t, cap, P, rows


def _run_noalloc(torch, B, fam, params, thresh, t, cap, stream):
    """One call; returns the inputs (kept alive) and the device memory the
    call itself took (free memory just before minus just after)."""
    d_seqs, d_off = B.device_inputs(fam, "cuda:0")
    lens = np.array([len(s) for s in fam], dtype=np.int32)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    B.posteriors_noalloc(d_seqs.data_ptr(), d_off.data_ptr(), lens, params, thresh,
                         {k: v.data_ptr() for k, v in t.items()}, cap, stream.cuda_stream)
    stream.synchronize()
    taken = free0 - torch.cuda.mem_get_info()[0]
    return (d_seqs, d_off), taken


def _plan_result(B, fam, params, thresh):
    """The plan form's outputs, every pair swept with its first sequence as
    rows (the allocation-free entry point never transposes a pair), so the
    two run the same arithmetic."""
    d_seqs, d_off = B.device_inputs(fam, "cuda:0")
    import torch
    lens = [len(s) for s in fam]
    orient = B.get_tuning()["orient"]
    B.set_tuning(orient=0)
    try:
        plan = B.Plan(lens, params, thresh, nnz_capacity=-1)
    finally:
        B.set_tuning(orient=orient)
    s = torch.cuda.current_stream()
    plan.run(d_seqs.data_ptr(), d_off.data_ptr(), s.cuda_stream)
    res = plan.download()
    plan.close()
    return res


def _compare(torch, t, res, P, rows):
    assert int(t["status"].item()) == 0
    h = {k: v.cpu().numpy() for k, v in t.items()}
    nnz = int(h["nnz_off"][P])
    assert nnz == res["nnz"]
    assert np.array_equal(h["pair_i"][:P], res["pair_i"]) and np.array_equal(h["pair_j"][:P], res["pair_j"])
    assert np.array_equal(h["row_off"], res["row_off"])
    assert np.array_equal(h["row_ptr"][:rows], res["row_ptr"])
    assert np.array_equal(h["nnz_off"], res["nnz_off"])
    assert np.array_equal(h["col"][:nnz], res["col"])
    # same kernels on the same pairs: bit-identical values
    assert np.array_equal(h["val"][:nnz], res["val"])
    assert np.array_equal(h["dist"][:P], res["dist"])
    assert np.array_equal(h["log_z"][:2 * P], res["log_z"])
    return nnz


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_plan_two_calls(B, params, prec):
    import torch
    from oracle import pair as oracle_pair
    p = B.make_params(params, prec)
    thresh = 0.01
    rng = np.random.default_rng(5)
    base = W.c1_family()
    # call 1: the C1 family plus a 300- and a 700-residue sequence (single-band
    # and banded kernel classes); call 2: five C1 sequences
    extra = [rng.integers(0, 20, size=L).astype(np.uint8) for L in (300, 700)]
    fams = [list(base) + extra, list(base[:5])]
    stream = torch.cuda.Stream()
    taken = []
    for call, fam in enumerate(fams):
        lens = np.array([len(s) for s in fam], dtype=np.int32)
        t, cap, P, rows = _outputs(torch, lens, thresh, B)
        torch.cuda.synchronize()
        _say("call %d (precision %d): %d sequences, %d pairs, capacity %d" % (call + 1, prec, len(fam), P, cap))
        keep, took = _run_noalloc(torch, B, fam, p, thresh, t, cap, stream)
        taken.append(took)
        _say("call %d: device memory taken by the call: %d bytes" % (call + 1, took))
        res = _plan_result(B, fam, p, thresh)
        nnz = _compare(torch, t, res, P, rows)
        _say("call %d: %d entries, equal to the plan form" % (call + 1, nnz))
        # and the bar against the oracle on a few pairs
        h = {k: v.cpu().numpy() for k, v in t.items()}
        for k in (0, P - 1):
            i, j = int(h["pair_i"][k]), int(h["pair_j"][k])
            orc = oracle_pair(fam[i], fam[j], params, per_model=False)
            a, b = h["nnz_off"][k], h["nnz_off"][k + 1]
            rp = h["row_ptr"][h["row_off"][k]:h["row_off"][k + 1]]
            r = np.repeat(np.arange(len(fam[i])), np.diff(rp))
            assert np.abs(h["val"][a:b] - orc["post"][r, h["col"][a:b]]).max(initial=0.0) <= 1e-5
            assert abs((1.0 - h["dist"][k]) - orc["ea"]) <= 1e-5
        del keep, t
    # the second call took no device memory (its workspace is the fixed array,
    # which the first call's module load brought in)
    assert taken[1] <= 0


def test_noalloc_empty_and_too_large(B, params):
    import torch
    p = B.make_params(params)
    t, cap, P, rows = _outputs(torch, np.array([40], np.int32), 0.01, B)
    stream = torch.cuda.Stream()
    fam = W.c1_family()[:1]
    _run_noalloc(torch, B, fam, p, 0.01, t, max(cap, 1), stream)
    assert int(t["status"].item()) == 0 and int(t["row_off"][0].item()) == 0 and int(t["nnz_off"][0].item()) == 0
    # a family whose bound-sized output pool cannot fit the fixed workspace
    lens = np.full(400, 400, dtype=np.int32)
    bound = B.output_bound(lens, 0.01)
    ptrs = {k: 4096 for k in B.NOALLOC_OUT_FIELDS}
    with pytest.raises(B.QpError) as e:
        B.posteriors_noalloc(4096, 4096, lens, p, 0.01, ptrs, bound, stream.cuda_stream)
    assert e.value.status == B.QP_ENOMEM and "QP_NOALLOC_SCRATCH_BYTES" in str(e.value)
