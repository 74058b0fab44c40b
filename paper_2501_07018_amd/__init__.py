"""Python binding of the gfx950 PDLP library (``include/pdlp.h``).

Argument marshalling only: every step of the solver runs in the HIP library
``libpdlp.so`` built in this directory.  There is no CPU fallback; loading
fails with an error when the library has not been built.

Functions carry the C names without the ``pdlp_`` prefix duplication kept,
e.g. ``pdlp_problem_create``; ``Problem`` is a small owner object around a
problem handle.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdlp.so")

PDLP_OK = 0
PDLP_ERR_INVALID_ARGUMENT = -1
PDLP_ERR_HIP = -2
PDLP_ERR_OUT_OF_MEMORY = -3
PDLP_ERR_STATE = -4
STATUS = {0: "OPTIMAL", 1: "ITERATION_LIMIT", 2: "TIME_LIMIT", 3: "NUMERICAL_ERROR",
          4: "PRIMAL_INFEASIBLE", 5: "DUAL_INFEASIBLE"}

D = C.POINTER(C.c_double)
I32 = C.POINTER(C.c_int32)


class PdlpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pdlp error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("eps_feas", C.c_double), ("eps_gap", C.c_double), ("max_iters", C.c_int64),
                ("time_limit", C.c_double), ("check_every", C.c_int32),
                ("ruiz_iters", C.c_int32), ("pock_chambolle", C.c_int32), ("polish", C.c_int32),
                ("polish_first", C.c_int64), ("reduced_cost_mode", C.c_int32),
                ("adaptive_restarts", C.c_int32), ("beta_suff", C.c_double),
                ("beta_nec", C.c_double), ("beta_art", C.c_double), ("theta", C.c_double),
                ("eps_zero", C.c_double), ("red_exp", C.c_double), ("grow_exp", C.c_double),
                ("verbose", C.c_int32), ("profile", C.c_int32), ("reorder", C.c_int32),
                ("detect_infeasibility", C.c_int32), ("eps_infeasible", C.c_double),
                ("restart_period", C.c_int64), ("fixed_step_size", C.c_double),
                ("fixed_primal_weight", C.c_double), ("graphs", C.c_int32),
                ("stream_block", C.c_int32), ("sorted_gathers", C.c_int32),
                ("segmented_gathers", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("x", D), ("y", D), ("r", D), ("status", C.c_int32), ("polished", C.c_int32),
                ("iterations", C.c_int64), ("attempts", C.c_int64), ("kkt_passes", C.c_int64),
                ("restarts", C.c_int64), ("restarts_i", C.c_int64), ("restarts_ii", C.c_int64),
                ("restarts_iii", C.c_int64), ("polish_attempts", C.c_int64),
                ("polish_iters", C.c_int64), ("primal_obj", C.c_double),
                ("dual_obj", C.c_double), ("rel_gap", C.c_double),
                ("primal_res_abs", C.c_double), ("primal_res_rel", C.c_double),
                ("dual_res_abs", C.c_double), ("dual_res_rel", C.c_double),
                ("omega", C.c_double), ("eta", C.c_double), ("seconds", C.c_double),
                ("seconds_setup", C.c_double), ("certificate", C.c_int32),
                ("reserved", C.c_int32), ("certificate_objective", C.c_double),
                ("certificate_residual", C.c_double)]


class IterInfo(C.Structure):
    _fields_ = [("k", C.c_int64), ("t", C.c_int64), ("n_outer", C.c_int64),
                ("attempts", C.c_int64), ("kkt_passes", C.c_int64),
                ("restarts_i", C.c_int64), ("restarts_ii", C.c_int64),
                ("restarts_iii", C.c_int64), ("omega", C.c_double), ("eta_hat", C.c_double),
                ("last_eta", C.c_double), ("last_eta_bar", C.c_double), ("seta", C.c_double),
                ("mu_ref", C.c_double), ("mu_c_prev", C.c_double)]


class KernelStats(C.Structure):
    _fields_ = [("dual_launches", C.c_int64), ("primal_launches", C.c_int64),
                ("attempts", C.c_int64), ("dual_ms", C.c_double), ("primal_ms", C.c_double),
                ("decide_ms", C.c_double), ("standalone_primal_ms", C.c_double),
                ("check_ms", C.c_double), ("primal_gather_ms", C.c_double)]


class DeviceRates(C.Structure):
    _fields_ = [("copy_gbs", C.c_double), ("gather_gps", C.c_double),
                ("gather_l2_gps", C.c_double)]


class BatchStats(C.Structure):
    _fields_ = [("rounds", C.c_int64), ("attempt_launches", C.c_int64),
                ("max_iterations", C.c_int64), ("total_iterations", C.c_int64),
                ("gap_evals", C.c_int64), ("gap_steps", C.c_int64), ("gap_capped", C.c_int64),
                ("seconds", C.c_double), ("setup_seconds", C.c_double),
                ("step_seconds", C.c_double), ("check_seconds", C.c_double)]


class UnrollStats(C.Structure):
    _fields_ = [("K", C.c_int64), ("ckpt", C.c_int64), ("restarts", C.c_int64),
                ("forward_seconds", C.c_double), ("replay_seconds", C.c_double),
                ("backward_seconds", C.c_double), ("backward_replay_seconds", C.c_double),
                ("backward_reverse_seconds", C.c_double), ("tangent_seconds", C.c_double)]


class StateBlob(C.Structure):
    _fields_ = [(k, D) for k in ("x", "y", "ax", "aty", "x0", "y0", "sx", "sy")] + \
               [(k, C.c_double) for k in ("seta", "omega", "eta_hat", "mu_ref", "mu_c_prev",
                                          "last_eta")] + \
               [(k, C.c_int64) for k in ("k", "t", "n_outer", "attempts", "kkt_passes",
                                         "restarts_i", "restarts_ii", "restarts_iii")]


_lib = None

EXPORTS = ("pdlp_problem_create", "pdlp_problem_create_device", "pdlp_problem_destroy",
           "pdlp_problem_dims", "pdlp_problem_schedule",
           "pdlp_problem_get_scaled", "pdlp_spmv", "pdlp_params_default", "pdlp_solve",
           "pdlp_state_create", "pdlp_state_destroy", "pdlp_iterate_k", "pdlp_state_get",
           "pdlp_state_set", "pdlp_norm_gap", "pdlp_last_error", "pdlp_state_solve",
           "pdlp_state_kernel_stats", "pdlp_measure_device_rates", "pdlp_batch_create",
           "pdlp_batch_destroy", "pdlp_batch_dims", "pdlp_batch_solve", "pdlp_batch_get_stats",
           "pdlp_unroll_create", "pdlp_unroll_destroy", "pdlp_unroll_set_data",
           "pdlp_unroll_forward", "pdlp_unroll_replay", "pdlp_unroll_backward",
           "pdlp_unroll_get_tape", "pdlp_unroll_get_stats", "pdlp_spmv_noalloc",
           "pdlp_unroll_tangent", "pdlp_unroll_set_data_device", "pdlp_unroll_forward_device",
           "pdlp_unroll_backward_device", "pdlp_unroll_tangent_device",
           "pdlp_batch_create_device", "pdlp_unroll_create_device")


def lib() -> C.CDLL:
    """Load libpdlp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_2501_07018_amd/build.py` (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.pdlp_problem_create.argtypes = [C.c_int32, C.c_int32, C.c_int64, I32, I32, D, D, D, D, D, D,
                                      C.c_double, C.POINTER(Params), vp, C.POINTER(vp)]
    L.pdlp_problem_create_device.argtypes = [C.c_int32, C.c_int32, C.c_int64] + [vp] * 8 + \
        [C.c_double, C.POINTER(Params), vp, C.POINTER(vp)]
    L.pdlp_problem_destroy.argtypes = [vp]
    L.pdlp_problem_destroy.restype = None
    L.pdlp_problem_dims.argtypes = [vp, I32, I32, C.POINTER(C.c_int64)]
    L.pdlp_problem_schedule.argtypes = [vp, I32, I32]
    L.pdlp_problem_get_scaled.argtypes = [vp, D, D, D, D, D, D, D, D]
    L.pdlp_spmv.argtypes = [vp, C.c_int32, C.c_int32, D, D, C.c_int32, D]
    L.pdlp_spmv_noalloc.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, vp]
    L.pdlp_params_default.argtypes = [C.POINTER(Params)]
    L.pdlp_params_default.restype = None
    L.pdlp_solve.argtypes = [vp, C.POINTER(Params), D, D, C.POINTER(Result)]
    L.pdlp_state_create.argtypes = [vp, C.POINTER(Params), C.POINTER(vp)]
    L.pdlp_state_destroy.argtypes = [vp]
    L.pdlp_state_destroy.restype = None
    L.pdlp_iterate_k.argtypes = [vp, C.c_int64, C.POINTER(IterInfo)]
    L.pdlp_state_get.argtypes = [vp, C.POINTER(StateBlob)]
    L.pdlp_state_set.argtypes = [vp, C.POINTER(StateBlob)]
    L.pdlp_norm_gap.argtypes = [vp, D, D, D, D, D, D, C.c_double, D]
    L.pdlp_state_solve.argtypes = [vp, C.c_int64, C.POINTER(Result)]
    L.pdlp_state_kernel_stats.argtypes = [vp, C.POINTER(KernelStats), C.c_int32]
    L.pdlp_measure_device_rates.argtypes = [C.c_int64, C.c_int64, C.POINTER(DeviceRates)]
    I64 = C.POINTER(C.c_int64)
    L.pdlp_batch_create.argtypes = [C.c_int32, I32, I32, I64, I32, I32, D, D, D, D, D, D, D,
                                    C.POINTER(Params), vp, C.POINTER(vp)]
    L.pdlp_batch_destroy.argtypes = [vp]
    L.pdlp_batch_destroy.restype = None
    L.pdlp_batch_dims.argtypes = [vp, I32, I64, I64, I64]
    L.pdlp_batch_solve.argtypes = [vp, C.POINTER(Params), C.POINTER(Result), D, D, D]
    L.pdlp_batch_get_stats.argtypes = [vp, C.POINTER(BatchStats)]
    L.pdlp_unroll_create.argtypes = [C.c_int32, I32, I32, I64, I32, I32, D, D, D, D, D, D,
                                     C.POINTER(Params), vp, C.POINTER(vp)]
    L.pdlp_unroll_destroy.argtypes = [vp]
    L.pdlp_unroll_destroy.restype = None
    L.pdlp_unroll_set_data.argtypes = [vp, D, D, D, D]
    L.pdlp_unroll_forward.argtypes = [vp, C.POINTER(Params), C.c_int64, C.c_int32, D]
    L.pdlp_unroll_replay.argtypes = [vp, D, I64]
    L.pdlp_unroll_backward.argtypes = [vp, D, D, D, D, D]
    L.pdlp_unroll_tangent.argtypes = [vp, D, D, D, D, D]
    L.pdlp_unroll_set_data_device.argtypes = [vp, vp, vp, vp, vp, vp]
    L.pdlp_unroll_forward_device.argtypes = [vp, C.POINTER(Params), C.c_int64, C.c_int32, vp, vp]
    L.pdlp_unroll_backward_device.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.pdlp_unroll_tangent_device.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.pdlp_batch_create_device.argtypes = [C.c_int32, I32, I32, I64] + [vp] * 8 + \
        [D, C.POINTER(Params), vp, C.POINTER(vp)]
    L.pdlp_unroll_create_device.argtypes = [C.c_int32, I32, I32, I64] + [vp] * 8 + \
        [C.POINTER(Params), vp, C.POINTER(vp)]
    L.pdlp_unroll_get_tape.argtypes = [vp, D, D, I32]
    L.pdlp_unroll_get_stats.argtypes = [vp, C.POINTER(UnrollStats)]
    L.pdlp_last_error.argtypes = []
    L.pdlp_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(rc):
    if rc != PDLP_OK:
        raise PdlpError(rc, lib().pdlp_last_error().decode())


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def pdlp_params_default(**over) -> Params:
    p = Params()
    lib().pdlp_params_default(C.byref(p))
    for k, v in over.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def pdlp_problem_create(m, n, row_ptr, col, val, c, lc, uc, lv, uv, obj_offset=0.0,
                        params: Params | None = None, stream=None):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    arrs = [_f64(a) for a in (val, c, lc, uc, lv, uv)]
    h = C.c_void_p()
    rc = lib().pdlp_problem_create(int(m), int(n), int(rp[-1]) if rp.size else 0,
                                   rp.ctypes.data_as(I32), cl.ctypes.data_as(I32),
                                   *[_d(a) for a in arrs], float(obj_offset),
                                   C.byref(params) if params is not None else None,
                                   stream, C.byref(h))
    _check(rc)
    return h


def pdlp_problem_create_device(m, n, nnz, row_ptr, col, val, c, lc, uc, lv, uv, obj_offset=0.0,
                               params: Params | None = None, stream=None):
    """Device-memory variant: each array argument is the integer address of
    int32 (row_ptr, col) or float64 (the others) storage in GPU memory."""
    h = C.c_void_p()
    ptrs = [C.c_void_p(int(a)) for a in (row_ptr, col, val, c, lc, uc, lv, uv)]
    rc = lib().pdlp_problem_create_device(int(m), int(n), int(nnz), *ptrs, float(obj_offset),
                                          C.byref(params) if params is not None else None,
                                          stream, C.byref(h))
    _check(rc)
    return h


def pdlp_problem_destroy(h):
    lib().pdlp_problem_destroy(h)


def pdlp_problem_dims(h):
    m, n, nnz = C.c_int32(), C.c_int32(), C.c_int64()
    _check(lib().pdlp_problem_dims(h, C.byref(m), C.byref(n), C.byref(nnz)))
    return m.value, n.value, nnz.value


def pdlp_problem_get_scaled(h) -> dict:
    m, n, nnz = pdlp_problem_dims(h)
    out = {"d1": np.empty(m), "d2": np.empty(n), "val": np.empty(nnz), "c": np.empty(n),
           "lc": np.empty(m), "uc": np.empty(m), "lv": np.empty(n), "uv": np.empty(n)}
    _check(lib().pdlp_problem_get_scaled(h, *[_d(out[k]) for k in
                                              ("d1", "d2", "val", "c", "lc", "uc", "lv", "uv")]))
    return out


def pdlp_spmv(h, x, transpose=False, scaled=True, repeat=1):
    m, n, _ = pdlp_problem_dims(h)
    x = _f64(x)
    out = np.empty(n if transpose else m)
    ms = C.c_double()
    _check(lib().pdlp_spmv(h, int(bool(transpose)), int(bool(scaled)), _d(x), _d(out),
                           int(repeat), C.byref(ms)))
    return out, ms.value


def pdlp_spmv_noalloc(h, x_dev, out_dev, transpose=False, scaled=True, stream=None):
    """Product on device buffers (integer addresses) with no allocation; asynchronous on
    `stream` (a HIP stream handle, None for the problem's stream)."""
    _check(lib().pdlp_spmv_noalloc(h, int(bool(transpose)), int(bool(scaled)),
                                   C.c_void_p(x_dev), C.c_void_p(out_dev),
                                   C.c_void_p(stream) if stream else None))


def pdlp_solve(h, params: Params | None = None, x0=None, y0=None) -> dict:
    m, n, _ = pdlp_problem_dims(h)
    x = np.empty(n)
    y = np.empty(m)
    r = np.empty(n)
    res = Result()
    res.x, res.y, res.r = _d(x), _d(y), _d(r)
    x0 = None if x0 is None else _f64(x0)
    y0 = None if y0 is None else _f64(y0)
    _check(lib().pdlp_solve(h, C.byref(params) if params is not None else None, _d(x0), _d(y0),
                            C.byref(res)))
    d = {f: getattr(res, f) for f, _ in Result._fields_ if f not in ("x", "y", "r")}
    d["status_name"] = STATUS.get(d["status"], str(d["status"]))
    d["x"], d["y"], d["r"] = x, y, r
    return d


def pdlp_state_create(h, params: Params | None = None):
    s = C.c_void_p()
    _check(lib().pdlp_state_create(h, C.byref(params) if params is not None else None, C.byref(s)))
    return s


def pdlp_state_destroy(s):
    lib().pdlp_state_destroy(s)


def pdlp_iterate_k(s, k) -> dict:
    info = IterInfo()
    _check(lib().pdlp_iterate_k(s, int(k), C.byref(info)))
    return {f: getattr(info, f) for f, _ in IterInfo._fields_}


def pdlp_state_solve(s, k, m=None, n=None, want_solution=False) -> dict:
    res = Result()
    arrs = {}
    if want_solution:
        arrs = {"x": np.empty(n), "y": np.empty(m), "r": np.empty(n)}
        res.x, res.y, res.r = _d(arrs["x"]), _d(arrs["y"]), _d(arrs["r"])
    _check(lib().pdlp_state_solve(s, int(k), C.byref(res)))
    d = {f: getattr(res, f) for f, _ in Result._fields_ if f not in ("x", "y", "r")}
    d["status_name"] = STATUS.get(d["status"], str(d["status"]))
    d.update(arrs)
    return d


def pdlp_state_kernel_stats(s, reset=False) -> dict:
    st = KernelStats()
    _check(lib().pdlp_state_kernel_stats(s, C.byref(st), int(bool(reset))))
    return {f: getattr(st, f) for f, _ in KernelStats._fields_}


def pdlp_state_get(s, m, n) -> dict:
    arrs = {k: np.empty(n) for k in ("x", "aty", "x0", "sx")}
    arrs.update({k: np.empty(m) for k in ("y", "ax", "y0", "sy")})
    b = StateBlob(*[_d(arrs[k]) for k in ("x", "y", "ax", "aty", "x0", "y0", "sx", "sy")])
    _check(lib().pdlp_state_get(s, C.byref(b)))
    for f, _ in StateBlob._fields_[8:]:
        arrs[f] = getattr(b, f)
    return arrs


def pdlp_state_set(s, blob: dict):
    arrs = {k: _f64(blob[k]) for k in ("x", "y", "ax", "aty", "x0", "y0", "sx", "sy")}
    b = StateBlob(*[_d(arrs[k]) for k in ("x", "y", "ax", "aty", "x0", "y0", "sx", "sy")])
    for f, _ in StateBlob._fields_[8:]:
        setattr(b, f, blob[f])
    _check(lib().pdlp_state_set(s, C.byref(b)))


def pdlp_norm_gap(h, x, y, ax, aty, xr, yr, omega) -> float:
    mu = C.c_double()
    x, y, ax, aty, xr, yr = map(_f64, (x, y, ax, aty, xr, yr))
    _check(lib().pdlp_norm_gap(h, _d(x), _d(y), _d(ax), _d(aty), _d(xr), _d(yr), float(omega),
                               C.byref(mu)))
    return mu.value


def pdlp_measure_device_rates(copy_bytes=2 << 30, gather_len=25_000_000) -> dict:
    r = DeviceRates()
    _check(lib().pdlp_measure_device_rates(int(copy_bytes), int(gather_len), C.byref(r)))
    return {f: getattr(r, f) for f, _ in DeviceRates._fields_}


def pdlp_batch_create(lps, params: Params | None = None, stream=None):
    """Create a batch from a sequence of objects with CSR fields (as Problem)."""
    count = len(lps)
    m = np.array([lp.m for lp in lps], dtype=np.int32)
    n = np.array([lp.n for lp in lps], dtype=np.int32)
    nnz = np.array([int(lp.row_ptr[-1]) if len(lp.row_ptr) else 0 for lp in lps], dtype=np.int64)
    rp = np.ascontiguousarray(np.concatenate([np.asarray(lp.row_ptr, dtype=np.int32)
                                              for lp in lps]), dtype=np.int32)
    cl = np.ascontiguousarray(np.concatenate([np.asarray(lp.col, dtype=np.int32) for lp in lps]),
                              dtype=np.int32)
    cat = {k: _f64(np.concatenate([np.asarray(getattr(lp, k), dtype=np.float64) for lp in lps]))
           for k in ("val", "c", "lc", "uc", "lv", "uv")}
    off = _f64([getattr(lp, "obj_offset", 0.0) for lp in lps])
    h = C.c_void_p()
    rc = lib().pdlp_batch_create(int(count), m.ctypes.data_as(I32), n.ctypes.data_as(I32),
                                 nnz.ctypes.data_as(C.POINTER(C.c_int64)), rp.ctypes.data_as(I32),
                                 cl.ctypes.data_as(I32),
                                 *[_d(cat[k]) for k in ("val", "c", "lc", "uc", "lv", "uv")],
                                 _d(off), C.byref(params) if params is not None else None,
                                 stream, C.byref(h))
    _check(rc)
    return h


def pdlp_batch_destroy(h):
    lib().pdlp_batch_destroy(h)


def pdlp_batch_dims(h):
    cnt, m, n, nnz = C.c_int32(), C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().pdlp_batch_dims(h, C.byref(cnt), C.byref(m), C.byref(n), C.byref(nnz)))
    return cnt.value, m.value, n.value, nnz.value


def pdlp_batch_solve(h, params: Params | None = None, want_solution=True):
    """Solve every instance; returns (results, x, y, r) with x, y, r concatenated
    in instance order (None unless want_solution)."""
    cnt, m, n, _ = pdlp_batch_dims(h)
    res = (Result * cnt)()
    x = y = r = None
    if want_solution:
        x, y, r = np.empty(n), np.empty(m), np.empty(n)
    _check(lib().pdlp_batch_solve(h, C.byref(params) if params is not None else None, res,
                                  _d(x), _d(y), _d(r)))
    out = []
    for i in range(cnt):
        d = {f: getattr(res[i], f) for f, _ in Result._fields_ if f not in ("x", "y", "r")}
        d["status_name"] = STATUS.get(d["status"], str(d["status"]))
        out.append(d)
    return out, x, y, r


def pdlp_batch_get_stats(h) -> dict:
    st = BatchStats()
    _check(lib().pdlp_batch_get_stats(h, C.byref(st)))
    return {f: getattr(st, f) for f, _ in BatchStats._fields_}


def _batch_tensors(m, n, nnz, ts):
    """Sizes as host arrays and the device addresses of the eight data tensors
    (row_ptr, col, val, c, lc, uc, lv, uv) of a batch in GPU memory; checks
    dtypes and lengths before anything is handed to the library."""
    import torch
    m = np.ascontiguousarray(m, dtype=np.int32)
    n = np.ascontiguousarray(n, dtype=np.int32)
    nnz = np.ascontiguousarray(nnz, dtype=np.int64)
    if not (m.ndim == n.ndim == nnz.ndim == 1) or not (len(m) == len(n) == len(nnz) >= 1):
        raise ValueError("m, n and nnz must be 1-D with one entry per instance")
    if (m < 0).any() or (n < 1).any() or (nnz < 0).any():
        raise ValueError("need m >= 0, n >= 1 and nnz >= 0 for every instance")
    M, N, NZ = int(m.sum()), int(n.sum()), int(nnz.sum())
    want = {"row_ptr": M + len(m), "col": NZ, "val": NZ, "c": N, "lc": M, "uc": M,
            "lv": N, "uv": N}
    for i, (name, t) in enumerate(zip(want, ts)):
        dt = torch.int32 if i < 2 else torch.float64
        if t.dtype != dt or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("tensors must be contiguous CUDA tensors: int32 row_ptr and col, "
                             "float64 val, c, lc, uc, lv, uv")
        if t.numel() != want[name]:
            raise ValueError(f"{name} has {t.numel()} elements, expected {want[name]}")
    return m, n, nnz, [_vp(t.data_ptr()) for t in ts]


class Batch:
    """Owner of a batch handle; solve() returns per-instance result dicts with
    the instance's x, y, r split out of the concatenated outputs."""

    def __init__(self, lps, params: Params | None = None, stream=None):
        self.m = [int(lp.m) for lp in lps]
        self.n = [int(lp.n) for lp in lps]
        self.h = pdlp_batch_create(lps, params, stream)

    @classmethod
    def from_tensors(cls, m, n, nnz, row_ptr, col, val, c, lc, uc, lv, uv, obj_offset=None,
                     params: Params | None = None) -> "Batch":
        """Create from torch tensors in GPU memory (the instances' arrays
        concatenated as for pdlp_batch_create), read on the current torch
        stream; m, n, nnz and obj_offset are host sequences."""
        import torch
        m, n, nnz, ptrs = _batch_tensors(m, n, nnz, (row_ptr, col, val, c, lc, uc, lv, uv))
        off = None if obj_offset is None else _f64(obj_offset)
        if off is not None and len(off) != len(m):
            raise ValueError("obj_offset needs one entry per instance")
        self = cls.__new__(cls)
        self.m, self.n = [int(v) for v in m], [int(v) for v in n]
        self.h = None
        h = C.c_void_p()
        _check(lib().pdlp_batch_create_device(
            len(m), m.ctypes.data_as(I32), n.ctypes.data_as(I32),
            nnz.ctypes.data_as(C.POINTER(C.c_int64)), *ptrs, _d(off),
            C.byref(params) if params is not None else None,
            C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(h)))
        self.h = h
        return self

    def solve(self, params: Params | None = None, want_solution=True) -> list:
        res, x, y, r = pdlp_batch_solve(self.h, params, want_solution)
        if want_solution:
            co = np.concatenate([[0], np.cumsum(self.n)])
            ro = np.concatenate([[0], np.cumsum(self.m)])
            for i, d in enumerate(res):
                d["x"] = x[co[i]:co[i + 1]]
                d["r"] = r[co[i]:co[i + 1]]
                d["y"] = y[ro[i]:ro[i + 1]]
        return res

    def stats(self) -> dict:
        return pdlp_batch_get_stats(self.h)

    def close(self):
        if self.h:
            pdlp_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _pack(lps):
    m = np.array([lp.m for lp in lps], dtype=np.int32)
    n = np.array([lp.n for lp in lps], dtype=np.int32)
    nnz = np.array([int(lp.row_ptr[-1]) if len(lp.row_ptr) else 0 for lp in lps], dtype=np.int64)
    rp = np.ascontiguousarray(np.concatenate([np.asarray(lp.row_ptr, dtype=np.int32)
                                              for lp in lps]), dtype=np.int32)
    cl = np.ascontiguousarray(np.concatenate([np.asarray(lp.col, dtype=np.int32) for lp in lps]),
                              dtype=np.int32)
    cat = {k: _f64(np.concatenate([np.asarray(getattr(lp, k), dtype=np.float64) for lp in lps]))
           for k in ("val", "c", "lc", "uc", "lv", "uv")}
    return m, n, nnz, rp, cl, cat


def _vp(a):
    return None if a is None else C.c_void_p(int(a))


class Unroll:
    """Owner of a pdlp_unroll handle: the differentiable K-step map over a batch.

    Arrays are concatenated over instances in instance order (x, c: sum n;
    lc, uc: sum m; val: sum nnz in each instance's CSR order)."""

    def __init__(self, lps, params: Params | None = None, stream=None):
        self.count = len(lps)
        m, n, nnz, rp, cl, cat = _pack(lps)
        self.m, self.n, self.nnz = m, n, nnz
        self.M, self.N, self.NZ = int(m.sum()), int(n.sum()), int(nnz.sum())
        self.h = C.c_void_p()
        _check(lib().pdlp_unroll_create(int(self.count), m.ctypes.data_as(I32),
                                        n.ctypes.data_as(I32),
                                        nnz.ctypes.data_as(C.POINTER(C.c_int64)),
                                        rp.ctypes.data_as(I32), cl.ctypes.data_as(I32),
                                        *[_d(cat[k]) for k in ("val", "c", "lc", "uc", "lv", "uv")],
                                        C.byref(params) if params is not None else None, stream,
                                        C.byref(self.h)))
        self.K = None

    @classmethod
    def from_tensors(cls, m, n, nnz, row_ptr, col, val, c, lc, uc, lv, uv,
                     params: Params | None = None) -> "Unroll":
        """Create from torch tensors in GPU memory (laid out as for Batch), read
        on the current torch stream; m, n and nnz are host sequences."""
        import torch
        m, n, nnz, ptrs = _batch_tensors(m, n, nnz, (row_ptr, col, val, c, lc, uc, lv, uv))
        self = cls.__new__(cls)
        self.count = len(m)
        self.m, self.n, self.nnz = m, n, nnz
        self.M, self.N, self.NZ = int(m.sum()), int(n.sum()), int(nnz.sum())
        self.h = C.c_void_p()
        self.K = None
        _check(lib().pdlp_unroll_create_device(
            self.count, m.ctypes.data_as(I32), n.ctypes.data_as(I32),
            nnz.ctypes.data_as(C.POINTER(C.c_int64)), *ptrs,
            C.byref(params) if params is not None else None,
            C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(self.h)))
        return self

    def set_data(self, c=None, lc=None, uc=None, val=None):
        arrs = [None if a is None else _f64(a) for a in (c, lc, uc, val)]
        _check(lib().pdlp_unroll_set_data(self.h, *[_d(a) for a in arrs]))

    def forward(self, K, ckpt=25, params: Params | None = None):
        x = np.empty(self.N)
        _check(lib().pdlp_unroll_forward(self.h, C.byref(params) if params is not None else None,
                                         int(K), int(ckpt), _d(x)))
        self.K = int(K)
        return x

    def replay(self):
        x = np.empty(self.N)
        sig = np.empty(self.count, dtype=np.int64)
        _check(lib().pdlp_unroll_replay(self.h, _d(x), sig.ctypes.data_as(C.POINTER(C.c_int64))))
        return x, sig

    def backward(self, gx) -> dict:
        gx = _f64(gx)
        out = {"c": np.empty(self.N), "lc": np.empty(self.M), "uc": np.empty(self.M),
               "val": np.empty(self.NZ)}
        _check(lib().pdlp_unroll_backward(self.h, _d(gx), _d(out["c"]), _d(out["lc"]),
                                          _d(out["uc"]), _d(out["val"])))
        return out

    def tangent(self, dc=None, dlc=None, duc=None, dval=None):
        """Directional derivative of x_K along a data direction (original units; None = 0)."""
        arrs = [None if a is None else _f64(a) for a in (dc, dlc, duc, dval)]
        dx = np.empty(self.N)
        _check(lib().pdlp_unroll_tangent(self.h, *[_d(a) for a in arrs], _d(dx)))
        return dx

    # device-memory variants: arguments are device addresses (int) or None
    def set_data_device(self, c=None, lc=None, uc=None, val=None, stream=None):
        _check(lib().pdlp_unroll_set_data_device(self.h, *[_vp(a) for a in (c, lc, uc, val)],
                                                 _vp(stream)))

    def forward_device(self, K, ckpt, x_ptr, params: Params | None = None, stream=None):
        _check(lib().pdlp_unroll_forward_device(
            self.h, C.byref(params) if params is not None else None, int(K), int(ckpt),
            _vp(x_ptr), _vp(stream)))
        self.K = int(K)

    def backward_device(self, gx_ptr, gc_ptr, glc_ptr, guc_ptr, gval_ptr, stream=None):
        _check(lib().pdlp_unroll_backward_device(
            self.h, *[_vp(a) for a in (gx_ptr, gc_ptr, glc_ptr, guc_ptr, gval_ptr)], _vp(stream)))

    def tangent_device(self, dc_ptr, dlc_ptr, duc_ptr, dval_ptr, dx_ptr, stream=None):
        _check(lib().pdlp_unroll_tangent_device(
            self.h, *[_vp(a) for a in (dc_ptr, dlc_ptr, duc_ptr, dval_ptr, dx_ptr)], _vp(stream)))

    def tape(self):
        K = self.K or 0
        eta = np.empty(self.count * K)
        omega = np.empty(self.count * K)
        rst = np.empty(self.count * K, dtype=np.int32)
        _check(lib().pdlp_unroll_get_tape(self.h, _d(eta), _d(omega), rst.ctypes.data_as(I32)))
        return (eta.reshape(self.count, K), omega.reshape(self.count, K),
                rst.reshape(self.count, K))

    def stats(self) -> dict:
        st = UnrollStats()
        _check(lib().pdlp_unroll_get_stats(self.h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in UnrollStats._fields_}

    def close(self):
        if self.h:
            lib().pdlp_unroll_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pdlp_last_error() -> str:
    return lib().pdlp_last_error().decode()


class Problem:
    """Owner of a problem handle created from an object with CSR fields
    (m, n, row_ptr, col, val, c, lc, uc, lv, uv, obj_offset)."""

    def __init__(self, lp, params: Params | None = None, stream=None):
        self.m, self.n = int(lp.m), int(lp.n)
        self.h = pdlp_problem_create(lp.m, lp.n, lp.row_ptr, lp.col, lp.val, lp.c, lp.lc, lp.uc,
                                     lp.lv, lp.uv, getattr(lp, "obj_offset", 0.0), params, stream)

    @classmethod
    def from_tensors(cls, m, n, row_ptr, col, val, c, lc, uc, lv, uv, obj_offset=0.0,
                     params: Params | None = None) -> "Problem":
        """Create from torch tensors in GPU memory (int32 row_ptr/col, float64
        others, contiguous), read on the current torch stream."""
        import torch
        ts = (row_ptr, col, val, c, lc, uc, lv, uv)
        for i, t in enumerate(ts):
            want = torch.int32 if i < 2 else torch.float64
            if t.dtype != want or not t.is_contiguous() or not t.is_cuda:
                raise ValueError("tensors must be contiguous CUDA tensors: int32 row_ptr and "
                                 "col, float64 val, c, lc, uc, lv, uv")
        m, n = int(m), int(n)
        if m < 0 or n < 0:
            raise ValueError("m and n must be >= 0")
        nnz = col.numel()
        want_len = {"row_ptr": m + 1, "col": nnz, "val": nnz, "c": n, "lc": m, "uc": m,
                    "lv": n, "uv": n}
        for name, t in zip(want_len, ts):
            if t.numel() != want_len[name]:
                raise ValueError(f"{name} has {t.numel()} elements, expected {want_len[name]} "
                                 f"(m={m}, n={n}, nnz={nnz})")
        self = cls.__new__(cls)
        self.m, self.n = m, n
        self.h = None
        self.h = pdlp_problem_create_device(
            m, n, col.numel(), *[t.data_ptr() for t in ts], obj_offset, params,
            C.c_void_p(torch.cuda.current_stream().cuda_stream))
        return self

    def close(self):
        if self.h:
            pdlp_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, params: Params | None = None, x0=None, y0=None) -> dict:
        return pdlp_solve(self.h, params, x0, y0)

    def scaled(self) -> dict:
        return pdlp_problem_get_scaled(self.h)

    def schedule(self) -> dict:
        sb, med = C.c_int32(), C.c_int32()
        _check(lib().pdlp_problem_schedule(self.h, C.byref(sb), C.byref(med)))
        return {"stream_block": sb.value, "med_row": med.value}

    def spmv(self, x, transpose=False, scaled=True, repeat=1):
        return pdlp_spmv(self.h, x, transpose, scaled, repeat)

    def state(self, params: Params | None = None) -> "State":
        return State(self, params)


class State:
    def __init__(self, prob: Problem, params: Params | None = None):
        self.prob = prob
        self.s = pdlp_state_create(prob.h, params)

    def iterate(self, k) -> dict:
        return pdlp_iterate_k(self.s, k)

    def solve(self, k, want_solution=False) -> dict:
        return pdlp_state_solve(self.s, k, self.prob.m, self.prob.n, want_solution)

    def kernel_stats(self, reset=False) -> dict:
        return pdlp_state_kernel_stats(self.s, reset)

    def get(self) -> dict:
        return pdlp_state_get(self.s, self.prob.m, self.prob.n)

    def set(self, blob: dict):
        pdlp_state_set(self.s, blob)

    def close(self):
        if self.s:
            pdlp_state_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
