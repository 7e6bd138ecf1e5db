"""ctypes binding of ``libqp.so`` (the C ABI declared in ``include/qp.h``).

Argument marshalling only: every step of the posterior computation runs in
the library's gfx950 kernels.  Functions keep the C names.  If the library is
missing, importing this module raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqp.so")

QP_OK, QP_EINVAL, QP_ENOMEM, QP_EDEVICE, QP_EBUSY, QP_ETIMEDOUT, QP_ECANCELED, QP_ENOSPC = 0, -1, -2, -3, -4, -5, -6, -7
QP_FP32_SCALED, QP_FP64 = 0, 1
KERNEL_CLASSES = 12  # QP_KERNEL_CLASSES: 0..7 single band, 8..11 banded (5..8 rows per lane)
BANDED = 8           # tuning entry of the banded classes
STATUS_NAMES = {0: "QP_OK", -1: "QP_EINVAL", -2: "QP_ENOMEM", -3: "QP_EDEVICE", -4: "QP_EBUSY",
                -5: "QP_ETIMEDOUT", -6: "QP_ECANCELED", -7: "QP_ENOSPC"}


class QpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class qp_params(ctypes.Structure):
    _fields_ = [("joint", ctypes.c_double * 400), ("n_gap_classes", ctypes.c_int32),
                ("gap_open", ctypes.c_double * 2), ("gap_extend", ctypes.c_double * 2),
                ("score", ctypes.c_double * 400), ("pf_gap_open", ctypes.c_double),
                ("pf_gap_extend", ctypes.c_double), ("temperature", ctypes.c_double),
                ("w_hmm", ctypes.c_double), ("precision", ctypes.c_int32), ("alphabet", ctypes.c_int32)]


class qp_result(ctypes.Structure):
    _fields_ = [("n_seqs", ctypes.c_int32), ("n_pairs", ctypes.c_int64), ("total_rows", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("pair_i", ctypes.POINTER(ctypes.c_int32)),
                ("pair_j", ctypes.POINTER(ctypes.c_int32)), ("row_off", ctypes.POINTER(ctypes.c_int64)),
                ("row_ptr", ctypes.POINTER(ctypes.c_int32)), ("nnz_off", ctypes.POINTER(ctypes.c_int64)),
                ("col", ctypes.POINTER(ctypes.c_int32)), ("val", ctypes.POINTER(ctypes.c_float)),
                ("dist", ctypes.POINTER(ctypes.c_double)), ("log_z", ctypes.POINTER(ctypes.c_double)),
                ("device_ms", ctypes.c_double), ("thresh", ctypes.c_float)]


class qp_device_result(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_int64), ("total_rows", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("pair_i", ctypes.c_void_p), ("pair_j", ctypes.c_void_p), ("row_off", ctypes.c_void_p),
                ("row_ptr", ctypes.c_void_p), ("nnz_off", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("dist", ctypes.c_void_p), ("log_z", ctypes.c_void_p)]


class qp_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32), ("n_streams", ctypes.c_int32)]


class qp_request_times(ctypes.Structure):
    _fields_ = [("submit_s", ctypes.c_double), ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double),
                ("cells", ctypes.c_int64), ("launched_s", ctypes.c_double), ("device_s", ctypes.c_double)]


class qp_noalloc_out(ctypes.Structure):
    _fields_ = [("pair_i", ctypes.c_void_p), ("pair_j", ctypes.c_void_p), ("row_off", ctypes.c_void_p),
                ("row_ptr", ctypes.c_void_p), ("nnz_off", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("capacity", ctypes.c_int64), ("dist", ctypes.c_void_p),
                ("log_z", ctypes.c_void_p), ("status", ctypes.c_void_p)]


# every function the header declares: name -> (restype, argtypes)
_P = ctypes.POINTER
_u8pp = _P(_P(ctypes.c_uint8))
class qp_tuning(ctypes.Structure):
    _fields_ = [("rows_per_lane", ctypes.c_int32 * 8), ("waves_frac", ctypes.c_double * 9),
                ("recompute", ctypes.c_int32 * 9), ("concurrent_classes", ctypes.c_int32), ("orient", ctypes.c_int32)]


SIGNATURES = {
    "qp_version": (ctypes.c_int32, []),
    "qp_last_error": (ctypes.c_char_p, []),
    "qp_params_default": (None, [_P(qp_params)]),
    "qp_params_check": (ctypes.c_int, [_P(qp_params)]),
    "qp_posteriors": (ctypes.c_int, [_u8pp, _P(ctypes.c_int32), ctypes.c_int32, _P(qp_params), ctypes.c_float,
                                     _P(_P(qp_result))]),
    "qp_posteriors_pairs": (ctypes.c_int, [_u8pp, _P(ctypes.c_int32), ctypes.c_int32, _P(ctypes.c_int32),
                                           _P(ctypes.c_int32), ctypes.c_int64, _P(qp_params), ctypes.c_float,
                                           _P(_P(qp_result))]),
    "qp_result_free": (None, [_P(qp_result)]),
    "qp_plan_create": (ctypes.c_int, [_P(ctypes.c_int32), ctypes.c_int32, _P(ctypes.c_int32), _P(ctypes.c_int32),
                                      ctypes.c_int64, _P(qp_params), ctypes.c_float, ctypes.c_int64,
                                      _P(ctypes.c_void_p)]),
    "qp_plan_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "qp_plan_sync": (ctypes.c_int, [ctypes.c_void_p, _P(qp_device_result)]),
    "qp_plan_download": (ctypes.c_int, [ctypes.c_void_p, _P(_P(qp_result))]),
    "qp_plan_timing": (ctypes.c_int, [ctypes.c_void_p, _P(ctypes.c_double), _P(ctypes.c_double),
                                      _P(ctypes.c_int64), ctypes.c_int32]),
    "qp_plan_class_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _P(ctypes.c_double),
                                            _P(ctypes.c_int64), _P(ctypes.c_int64), _P(ctypes.c_int32)]),
    "qp_plan_set_graph": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "qp_plan_set_per_pair": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "qp_plan_device_bytes": (ctypes.c_int64, [ctypes.c_void_p]),
    "qp_plan_destroy": (None, [ctypes.c_void_p]),
    "qp_server_create": (ctypes.c_int, [_P(qp_server_config), _P(ctypes.c_void_p)]),
    "qp_server_submit": (ctypes.c_int, [ctypes.c_void_p, _u8pp, _P(ctypes.c_int32), ctypes.c_int32, _P(qp_params),
                                        ctypes.c_float, _P(ctypes.c_uint64)]),
    "qp_server_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, _P(_P(qp_result)),
                                      _P(qp_request_times)]),
    "qp_server_cancel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "qp_server_stats": (ctypes.c_int, [ctypes.c_void_p, _P(ctypes.c_int64), _P(ctypes.c_int64),
                                       _P(ctypes.c_int64), _P(ctypes.c_int64)]),
    "qp_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "qp_set_tuning": (ctypes.c_int, [_P(qp_tuning)]),
    "qp_output_bound": (ctypes.c_int, [_P(ctypes.c_int32), ctypes.c_int32, _P(ctypes.c_int32), _P(ctypes.c_int32),
                                       ctypes.c_int64, ctypes.c_float, _P(ctypes.c_int64)]),
    "qp_threshold_for_budget": (ctypes.c_int, [_P(ctypes.c_int32), ctypes.c_int32, _P(ctypes.c_int32),
                                               _P(ctypes.c_int32), ctypes.c_int64, ctypes.c_int64,
                                               _P(ctypes.c_float)]),
    "qp_guide_tree": (ctypes.c_int, [_P(ctypes.c_double), ctypes.c_int32, _P(ctypes.c_int32), _P(ctypes.c_double)]),
    "qp_tree_distance": (ctypes.c_int, [_P(ctypes.c_int32), ctypes.c_int32, _P(ctypes.c_int32)]),
    "qp_get_tuning": (ctypes.c_int, [_P(qp_tuning)]),
    "qp_posteriors_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, _P(ctypes.c_int32), ctypes.c_int32,
                                             _P(qp_params), ctypes.c_float, _P(qp_noalloc_out), ctypes.c_void_p]),
    "qp_relax_create": (ctypes.c_int, [_P(ctypes.c_int32), ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                       ctypes.c_double, ctypes.c_int32, ctypes.c_float, _P(ctypes.c_void_p)]),
    "qp_relax_run": (ctypes.c_int, [ctypes.c_void_p, _P(qp_device_result), ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_void_p]),
    "qp_relax_sync": (ctypes.c_int, [ctypes.c_void_p, _P(qp_device_result)]),
    "qp_relax_download": (ctypes.c_int, [ctypes.c_void_p, _P(_P(qp_result))]),
    "qp_relax_device_bytes": (ctypes.c_int64, [ctypes.c_void_p]),
    "qp_relax_destroy": (None, [ctypes.c_void_p]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libqp.so is not built (%s); run __graft_entry__.build() -- there is no CPU fallback"
                          % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(st: int):
    if st != QP_OK:
        raise QpError(st, lib.qp_last_error().decode(errors="replace"))


# tuning table written by the autotuner (paper_1512_07437_amd/autotune.py)
TUNING_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")


def set_tuning(rows_per_lane: Optional[Sequence[int]] = None, waves_frac: Optional[Sequence[float]] = None,
               recompute: Optional[Sequence[int]] = None, concurrent_classes: Optional[int] = None,
               orient: Optional[int] = None):
    """Process-wide tuning table for plans made afterwards (qp_set_tuning);
    entries left None keep their current values; None for all of them
    restores the default."""
    if (rows_per_lane is None and waves_frac is None and recompute is None and concurrent_classes is None
            and orient is None):
        _check(lib.qp_set_tuning(None))
        return
    t = get_tuning()
    r = list(t["rows_per_lane"] if rows_per_lane is None else rows_per_lane)
    w = list(t["waves_frac"] if waves_frac is None else waves_frac)
    c = list(t["recompute"] if recompute is None else recompute)
    v = qp_tuning()
    v.rows_per_lane[:] = [int(x) for x in r]
    v.waves_frac[:] = [float(x) for x in w]
    v.recompute[:] = [int(x) for x in c]
    v.concurrent_classes = int(t["concurrent_classes"] if concurrent_classes is None else concurrent_classes)
    v.orient = int(t["orient"] if orient is None else orient)
    _check(lib.qp_set_tuning(ctypes.byref(v)))


def get_tuning() -> Dict[str, list]:
    t = qp_tuning()
    _check(lib.qp_get_tuning(ctypes.byref(t)))
    return {"rows_per_lane": list(t.rows_per_lane), "waves_frac": list(t.waves_frac),
            "recompute": list(t.recompute), "concurrent_classes": int(t.concurrent_classes),
            "orient": int(t.orient)}


def load_tuning(path: str = TUNING_PATH) -> bool:
    """Apply a tuning table file if it exists; returns whether one was applied."""
    import json
    if not os.path.exists(path):
        return False
    with open(path) as f:
        d = json.load(f)
    set_tuning(d["rows_per_lane"], d["waves_frac"], d.get("recompute"), d.get("concurrent_classes"), d.get("orient"))
    return True


def _pairs_args(lens, pair_i, pair_j):
    lens = np.ascontiguousarray(lens, dtype=np.int32)
    if pair_i is None and pair_j is None:
        return lens, None, None, 0, (lens,)
    pi = np.ascontiguousarray(pair_i, dtype=np.int32)
    pj = np.ascontiguousarray(pair_j, dtype=np.int32)
    return lens, pi.ctypes.data_as(_P(ctypes.c_int32)), pj.ctypes.data_as(_P(ctypes.c_int32)), len(pi), (lens, pi, pj)


def output_bound(lens, thresh: float, pair_i=None, pair_j=None) -> int:
    """Entries the sparse output can reach at this threshold (no run exceeds it)."""
    lens, pi, pj, np_, keep = _pairs_args(lens, pair_i, pair_j)
    e = ctypes.c_int64()
    _check(lib.qp_output_bound(lens.ctypes.data_as(_P(ctypes.c_int32)), len(lens), pi, pj, np_,
                               ctypes.c_float(thresh), ctypes.byref(e)))
    return int(e.value)


def threshold_for_budget(lens, max_entries: int, pair_i=None, pair_j=None) -> float:
    """Smallest threshold whose output bound fits max_entries."""
    lens, pi, pj, np_, keep = _pairs_args(lens, pair_i, pair_j)
    t = ctypes.c_float()
    _check(lib.qp_threshold_for_budget(lens.ctypes.data_as(_P(ctypes.c_int32)), len(lens), pi, pj, np_,
                                       int(max_entries), ctypes.byref(t)))
    return float(t.value)


def guide_tree(dist, n: int):
    """Weighted UPGMA on the condensed distances (pair order of a result's
    ``dist``): (joins [n-1, 2] int32, heights [n-1] float64)."""
    d = np.ascontiguousarray(dist, dtype=np.float64)
    if d.shape != (n * (n - 1) // 2,):
        raise ValueError("dist must hold n(n-1)/2 values")
    joins = np.zeros((max(n - 1, 0), 2), dtype=np.int32)
    heights = np.zeros(max(n - 1, 0), dtype=np.float64)
    _check(lib.qp_guide_tree(d.ctypes.data_as(_P(ctypes.c_double)), int(n),
                             joins.ctypes.data_as(_P(ctypes.c_int32)), heights.ctypes.data_as(_P(ctypes.c_double))))
    return joins, heights


def tree_distance(joins, n: int) -> np.ndarray:
    """Tree-guided distance of every pair (pair order): nodes of the subtree
    under their lowest common ancestor."""
    j = np.ascontiguousarray(joins, dtype=np.int32).reshape(-1)
    if j.shape != (2 * max(n - 1, 0),):
        raise ValueError("joins must hold n-1 rows of two ids")
    out = np.zeros(n * (n - 1) // 2, dtype=np.int32)
    _check(lib.qp_tree_distance(j.ctypes.data_as(_P(ctypes.c_int32)), int(n), out.ctypes.data_as(_P(ctypes.c_int32))))
    return out


def qp_version() -> int:
    return int(lib.qp_version())


def qp_last_error() -> str:
    return lib.qp_last_error().decode(errors="replace")


def make_params(mp, precision: int = QP_FP32_SCALED) -> qp_params:
    """qp_params from a ``workload.ModelParams``."""
    p = qp_params()
    lib.qp_params_default(ctypes.byref(p))
    p.joint[:] = [float(v) for v in np.asarray(mp.joint, dtype=np.float64).reshape(400)]
    p.score[:] = [float(v) for v in np.asarray(mp.score, dtype=np.float64).reshape(400)]
    G = len(mp.gap_open)
    p.n_gap_classes = G
    for k in range(2):
        p.gap_open[k] = float(mp.gap_open[k]) if k < G else 0.0
        p.gap_extend[k] = float(mp.gap_extend[k]) if k < G else 0.0
    p.pf_gap_open = float(mp.pf_gap_open)
    p.pf_gap_extend = float(mp.pf_gap_extend)
    p.temperature = float(mp.temperature)
    p.w_hmm = float(mp.w_hmm)
    p.precision = int(precision)
    p.alphabet = int(getattr(mp, "alphabet", 20))
    return p


def qp_params_check(p: qp_params) -> int:
    return int(lib.qp_params_check(ctypes.byref(p)))


def _seq_array(seqs: Sequence[np.ndarray]):
    keep = [np.ascontiguousarray(s, dtype=np.uint8) for s in seqs]
    arr = (_P(ctypes.c_uint8) * max(1, len(keep)))()
    for i, s in enumerate(keep):
        arr[i] = s.ctypes.data_as(_P(ctypes.c_uint8))
    lens = np.asarray([len(s) for s in keep], dtype=np.int32)
    return keep, arr, lens


class _Owned:
    """Holds a library result; frees it once no array viewing it is left."""

    __slots__ = ("ptr",)

    def __init__(self, ptr):
        self.ptr = ptr

    def __del__(self):
        ptr, self.ptr = self.ptr, None
        if ptr is not None and lib is not None:
            try:
                lib.qp_result_free(ptr)
            except Exception:  # interpreter shutdown
                pass


def _view(owner: _Owned, ptr, count, dtype):
    """Zero-copy array over `count` elements at `ptr`, keeping `owner` alive."""
    if count <= 0:
        return np.zeros(0, dtype=dtype)
    dt = np.dtype(dtype)
    buf = (ctypes.c_char * (int(count) * dt.itemsize)).from_address(ctypes.cast(ptr, ctypes.c_void_p).value)
    buf._owner = owner
    return np.frombuffer(buf, dtype=dt, count=int(count))


def _take_result(out) -> Dict[str, np.ndarray]:
    """Result dict whose arrays view the library result `out` (a pointer
    from qp_posteriors / qp_plan_download / qp_server_wait) without copying
    it; the result is freed when the last of the arrays is."""
    owner = _Owned(out)
    try:
        r = out.contents
        P, rows, nnz = r.n_pairs, r.total_rows, r.nnz
        return dict(n_seqs=int(r.n_seqs), n_pairs=int(P), nnz=int(nnz), device_ms=float(r.device_ms),
                    thresh=float(r.thresh),
                    pair_i=_view(owner, r.pair_i, P, np.int32), pair_j=_view(owner, r.pair_j, P, np.int32),
                    row_off=_view(owner, r.row_off, P + 1, np.int64),
                    row_ptr=_view(owner, r.row_ptr, rows, np.int32),
                    nnz_off=_view(owner, r.nnz_off, P + 1, np.int64), col=_view(owner, r.col, nnz, np.int32),
                    val=_view(owner, r.val, nnz, np.float32), dist=_view(owner, r.dist, P, np.float64),
                    log_z=_view(owner, r.log_z, 2 * P, np.float64))
    finally:
        del owner  # the arrays hold it from here on


def qp_posteriors(seqs: Sequence[np.ndarray], params: qp_params, thresh: float) -> Dict[str, np.ndarray]:
    """All-pairs posteriors of one family (blocking)."""
    keep, arr, lens = _seq_array(seqs)
    out = _P(qp_result)()
    st = lib.qp_posteriors(arr, lens.ctypes.data_as(_P(ctypes.c_int32)), len(keep), ctypes.byref(params),
                           ctypes.c_float(thresh), ctypes.byref(out))
    _check(st)
    return _take_result(out)


def qp_posteriors_pairs(seqs: Sequence[np.ndarray], pair_i, pair_j, params: qp_params,
                        thresh: float) -> Dict[str, np.ndarray]:
    """Posteriors of an explicit pair list (blocking)."""
    keep, arr, lens = _seq_array(seqs)
    pi = np.ascontiguousarray(pair_i, dtype=np.int32)
    pj = np.ascontiguousarray(pair_j, dtype=np.int32)
    out = _P(qp_result)()
    st = lib.qp_posteriors_pairs(arr, lens.ctypes.data_as(_P(ctypes.c_int32)), len(keep),
                                 pi.ctypes.data_as(_P(ctypes.c_int32)), pj.ctypes.data_as(_P(ctypes.c_int32)),
                                 len(pi), ctypes.byref(params), ctypes.c_float(thresh), ctypes.byref(out))
    _check(st)
    return _take_result(out)


def pair_csr(res: Dict[str, np.ndarray], p: int):
    """(row_ptr, col, val) of pair p from a result dict."""
    rp = res["row_ptr"][res["row_off"][p]:res["row_off"][p + 1]]
    a, b = res["nnz_off"][p], res["nnz_off"][p + 1]
    return rp, res["col"][a:b], res["val"][a:b]


def pair_dense(res: Dict[str, np.ndarray], p: int, n_cols: int) -> np.ndarray:
    rp, c, v = pair_csr(res, p)
    m = len(rp) - 1
    d = np.zeros((m, n_cols), dtype=np.float64)
    for i in range(m):
        d[i, c[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
    return d


class Plan:
    """Device-resident plan (qp_plan_*): inputs are device buffers (torch
    tensors or hipMalloc'd memory), the stream any HIP stream; outputs stay on
    the device until downloaded.

    torch bundles its own HIP runtime; when torch and this library share a
    process, let torch initialize the GPU first (e.g. allocate a tensor before
    loading this module): torch's runtime does not initialize after another
    one has."""

    def __init__(self, lens: Sequence[int], params: qp_params, thresh: float, pair_i=None, pair_j=None,
                 nnz_capacity: int = 0):
        self._lens = np.ascontiguousarray(lens, dtype=np.int32)
        self.handle = ctypes.c_void_p()
        if pair_i is None:
            pi = pj = None
            npairs = 0
        else:
            self._pi = np.ascontiguousarray(pair_i, dtype=np.int32)
            self._pj = np.ascontiguousarray(pair_j, dtype=np.int32)
            pi = self._pi.ctypes.data_as(_P(ctypes.c_int32))
            pj = self._pj.ctypes.data_as(_P(ctypes.c_int32))
            npairs = len(self._pi)
        st = lib.qp_plan_create(self._lens.ctypes.data_as(_P(ctypes.c_int32)), len(self._lens), pi, pj, npairs,
                                ctypes.byref(params), ctypes.c_float(thresh), int(nnz_capacity),
                                ctypes.byref(self.handle))
        _check(st)

    def run(self, d_seqs_ptr: int, d_off_ptr: int, stream_ptr: int):
        _check(lib.qp_plan_run(self.handle, ctypes.c_void_p(d_seqs_ptr), ctypes.c_void_p(d_off_ptr),
                               ctypes.c_void_p(stream_ptr)))

    def sync(self) -> qp_device_result:
        r = qp_device_result()
        _check(lib.qp_plan_sync(self.handle, ctypes.byref(r)))
        return r

    def sync_status(self) -> int:
        """Status of the last run; on QP_ENOSPC, ``needed_nnz`` holds the
        entries it produced (a new plan needs at least that capacity)."""
        r = qp_device_result()
        st = int(lib.qp_plan_sync(self.handle, ctypes.byref(r)))
        self.needed_nnz = int(r.nnz) if st == QP_ENOSPC else 0
        return st

    def download(self) -> Dict[str, np.ndarray]:
        out = _P(qp_result)()
        _check(lib.qp_plan_download(self.handle, ctypes.byref(out)))
        return _take_result(out)

    def timing(self, reset: bool = False):
        k, p, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        _check(lib.qp_plan_timing(self.handle, ctypes.byref(k), ctypes.byref(p), ctypes.byref(n), int(reset)))
        return k.value, p.value, n.value

    def class_timing(self, cls: int):
        """(kernel_ms, pairs, cells, rows_per_lane) of one kernel class."""
        k, p, c, r = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _check(lib.qp_plan_class_timing(self.handle, int(cls), ctypes.byref(k), ctypes.byref(p), ctypes.byref(c),
                                        ctypes.byref(r)))
        return k.value, p.value, c.value, r.value

    def set_graph(self, on: bool):
        _check(lib.qp_plan_set_graph(self.handle, int(on)))

    def set_per_pair(self, on: bool):
        """Plain per-pair form (one launch per pair) instead of the batched one."""
        _check(lib.qp_plan_set_per_pair(self.handle, int(on)))

    def device_bytes(self) -> int:
        return int(lib.qp_plan_device_bytes(self.handle))

    def close(self):
        if self.handle:
            lib.qp_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


NOALLOC_OUT_FIELDS = ("pair_i", "pair_j", "row_off", "row_ptr", "nnz_off", "col", "val", "dist", "log_z", "status")


def posteriors_noalloc(d_seqs_ptr: int, d_off_ptr: int, lens, params: qp_params, thresh: float,
                       out_ptrs: Dict[str, int], capacity: int, stream_ptr: int):
    """qp_posteriors_noalloc: enqueue the allocation-free pipeline on a
    stream.  out_ptrs maps each qp_noalloc_out array name to a device
    pointer the caller owns (sizes as documented in include/qp.h); capacity
    is the entries col / val hold."""
    lens = np.ascontiguousarray(lens, dtype=np.int32)
    o = qp_noalloc_out()
    for name in NOALLOC_OUT_FIELDS:
        setattr(o, name, ctypes.c_void_p(int(out_ptrs[name])))
    o.capacity = int(capacity)
    _check(lib.qp_posteriors_noalloc(ctypes.c_void_p(d_seqs_ptr), ctypes.c_void_p(d_off_ptr),
                                     lens.ctypes.data_as(_P(ctypes.c_int32)), len(lens), ctypes.byref(params),
                                     ctypes.c_float(thresh), ctypes.byref(o), ctypes.c_void_p(stream_ptr)))


def device_result(n_pairs: int, total_rows: int, nnz: int, ptrs: Dict[str, int]) -> qp_device_result:
    """qp_device_result over caller-owned device arrays (pair_i, pair_j,
    row_off, row_ptr, nnz_off, col, val; dist and log_z optional)."""
    r = qp_device_result()
    r.n_pairs, r.total_rows, r.nnz = int(n_pairs), int(total_rows), int(nnz)
    for name in ("pair_i", "pair_j", "row_off", "row_ptr", "nnz_off", "col", "val", "dist", "log_z"):
        setattr(r, name, ctypes.c_void_p(int(ptrs.get(name, 0))))
    return r


class Relax:
    """Selective consistency on the device (qp_relax_*): relaxes the all-pairs
    CSR of a family through the third sequences the guide tree selects."""

    def __init__(self, lens: Sequence[int], tree_threshold: int, amplification: float, passes: int, thresh: float,
                 in_capacity: int = 0):
        self._lens = np.ascontiguousarray(lens, dtype=np.int32)
        self.handle = ctypes.c_void_p()
        _check(lib.qp_relax_create(self._lens.ctypes.data_as(_P(ctypes.c_int32)), len(self._lens),
                                   int(in_capacity), int(tree_threshold), float(amplification), int(passes),
                                   ctypes.c_float(thresh), ctypes.byref(self.handle)))

    def run(self, dev_in: qp_device_result, in_nnz: int, d_tdist_ptr: int, stream_ptr: int):
        self._in = dev_in  # read during the run
        _check(lib.qp_relax_run(self.handle, ctypes.byref(dev_in), int(in_nnz), ctypes.c_void_p(d_tdist_ptr),
                                ctypes.c_void_p(stream_ptr)))

    def sync(self) -> qp_device_result:
        r = qp_device_result()
        _check(lib.qp_relax_sync(self.handle, ctypes.byref(r)))
        return r

    def download(self) -> Dict[str, np.ndarray]:
        out = _P(qp_result)()
        _check(lib.qp_relax_download(self.handle, ctypes.byref(out)))
        return _take_result(out)

    def device_bytes(self) -> int:
        return int(lib.qp_relax_device_bytes(self.handle))

    def close(self):
        if self.handle:
            lib.qp_relax_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_inputs(seqs: Sequence[np.ndarray], device: str = "cuda:0"):
    """Concatenate a family into torch device tensors (codes, int64 offsets)."""
    import torch
    lens = np.asarray([len(s) for s in seqs], dtype=np.int64)
    off = np.zeros(len(seqs), dtype=np.int64)
    if len(seqs) > 1:
        off[1:] = np.cumsum(lens)[:-1]
    cat = np.concatenate([np.asarray(s, dtype=np.uint8) for s in seqs]) if len(seqs) else np.zeros(1, np.uint8)
    return torch.from_numpy(cat).to(device), torch.from_numpy(off).to(device)


class Server:
    """Serving loop (qp_server_*): submit families, wait for tickets."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 8, n_streams: int = 4):
        cfg = qp_server_config(int(hbm_budget_bytes), int(max_slots), int(n_streams))
        self.handle = ctypes.c_void_p()
        _check(lib.qp_server_create(ctypes.byref(cfg), ctypes.byref(self.handle)))

    def submit(self, seqs: Sequence[np.ndarray], params: qp_params, thresh: float) -> int:
        keep, arr, lens = _seq_array(seqs)
        t = ctypes.c_uint64()
        _check(lib.qp_server_submit(self.handle, arr, lens.ctypes.data_as(_P(ctypes.c_int32)), len(keep),
                                    ctypes.byref(params), ctypes.c_float(thresh), ctypes.byref(t)))
        return int(t.value)

    def wait(self, ticket: int, timeout_ms: int = -1):
        """Returns (result dict, times dict); raises QpError (QP_EBUSY /
        QP_ETIMEDOUT if not ready)."""
        out = _P(qp_result)()
        tm = qp_request_times()
        st = lib.qp_server_wait(self.handle, ctypes.c_uint64(ticket), int(timeout_ms), ctypes.byref(out),
                                ctypes.byref(tm))
        _check(st)
        res = _take_result(out)
        return res, dict(submit_s=tm.submit_s, admit_s=tm.admit_s, done_s=tm.done_s, cells=int(tm.cells),
                         launched_s=tm.launched_s, device_s=tm.device_s)

    def cancel(self, ticket: int) -> int:
        return int(lib.qp_server_cancel(self.handle, ctypes.c_uint64(ticket)))

    def stats(self):
        q, f, d, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.qp_server_stats(self.handle, ctypes.byref(q), ctypes.byref(f), ctypes.byref(d), ctypes.byref(b)))
        return dict(queued=q.value, in_flight=f.value, finished=d.value, bytes_in_use=b.value)

    def close(self):
        if self.handle:
            lib.qp_server_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# the autotuned table for gfx950, when one has been measured
load_tuning()
