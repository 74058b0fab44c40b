"""Python access to the FP64 CPU oracle (``pdlp_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this module; the product
package never does.  It shares no code with the GPU library: the only
common dependency is the seeded input generator package ``lpgen``.

The C sources follow the paper step by step (see the header comment of
``pdlp_oracle.c`` for the passage each function follows).  This module only
marshals numpy arrays into the C structs.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle_pdlp.so")
SRC = os.path.join(HERE, "pdlp_oracle.c")
SRCS = [SRC, os.path.join(HERE, "pdlp_oracle_unroll.c")]

D = C.POINTER(C.c_double)
I32 = C.POINTER(C.c_int32)


OMP_LIB_PATH = os.path.join(HERE, "liboracle_pdlp_omp.so")


def build(force: bool = False, threaded: bool = False) -> str:
    """Compile the oracle with gcc (-O2 -ffp-contract=off).  threaded: the
    OpenMP build of the same source used only by the all-cores CPU baseline
    (row-sharded products, Section 5 "Multithreading"); the plain build is
    the oracle the tests use."""
    path = OMP_LIB_PATH if threaded else LIB_PATH
    newest = max(os.path.getmtime(f) for f in SRCS + [os.path.join(HERE, "pdlp_oracle.h")])
    if force or not os.path.exists(path) or os.path.getmtime(path) < newest:
        tmp = path + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-Wall",
               "-Wno-unknown-pragmas", *(["-fopenmp"] if threaded else []), "-fPIC", "-shared", "-o", tmp, *SRCS, "-lm"]
        subprocess.run(cmd, check=True, cwd=HERE)
        os.replace(tmp, path)
    return path


class _LP(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("row_ptr", I32), ("col", I32),
                ("val", D), ("c", D), ("lc", D), ("uc", D), ("lv", D), ("uv", D)]


class _Params(C.Structure):
    _fields_ = [("eps_feas", C.c_double), ("eps_gap", C.c_double), ("max_iters", C.c_int64),
                ("check_every", C.c_int32), ("terminate", C.c_int32),
                ("beta_suff", C.c_double), ("beta_nec", C.c_double), ("beta_art", C.c_double),
                ("theta", C.c_double), ("eps_zero", C.c_double),
                ("red_exp", C.c_double), ("grow_exp", C.c_double),
                ("reduced_cost_mode", C.c_int32), ("polish", C.c_int32),
                ("polish_first", C.c_int64), ("fixed_step", C.c_int32),
                ("fixed_eta", C.c_double), ("adaptive_restarts", C.c_int32),
                ("detect_infeas", C.c_int32), ("eps_infeas", C.c_double),
                ("restart_period", C.c_int64), ("fixed_omega", C.c_double),
                ("signed_step_rule", C.c_int32)]


class _State(C.Structure):
    _fields_ = [("x", D), ("y", D), ("ax", D), ("aty", D), ("x0", D), ("y0", D),
                ("sx", D), ("sy", D), ("seta", C.c_double), ("omega", C.c_double),
                ("eta_hat", C.c_double), ("k", C.c_int64), ("t", C.c_int64),
                ("n_outer", C.c_int64), ("attempts", C.c_int64), ("kkt_passes", C.c_int64),
                ("mu_ref", C.c_double), ("mu_c_prev", C.c_double),
                ("restarts_i", C.c_int64), ("restarts_ii", C.c_int64),
                ("restarts_iii", C.c_int64), ("last_eta", C.c_double),
                ("last_eta_bar", C.c_double)]


class _Scratch(C.Structure):
    _fields_ = [(f"n{i}", D) for i in range(6)] + [(f"m{i}", D) for i in range(6)]


class _Unscale(C.Structure):
    _fields_ = [("orig", _LP), ("d1", D), ("d2", D), ("obj_offset", C.c_double)]


class _Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int64), ("attempts", C.c_int64),
                ("kkt_passes", C.c_int64), ("restarts", C.c_int64), ("restarts_i", C.c_int64),
                ("restarts_ii", C.c_int64), ("restarts_iii", C.c_int64),
                ("primal_obj", C.c_double), ("dual_obj", C.c_double), ("rel_gap", C.c_double),
                ("primal_res_abs", C.c_double), ("primal_res_rel", C.c_double),
                ("dual_res_abs", C.c_double), ("dual_res_rel", C.c_double),
                ("omega", C.c_double), ("eta", C.c_double),
                ("polish_attempts", C.c_int64), ("polish_iters", C.c_int64),
                ("polished", C.c_int32), ("cert_source", C.c_int32),
                ("cert_obj", C.c_double), ("cert_res", C.c_double)]


class _Tape(C.Structure):
    _fields_ = [("cap", C.c_int64), ("eta", D), ("omega", D), ("restart", I32)]


I64 = C.POINTER(C.c_int64)


class _Trace(C.Structure):
    _fields_ = [("cap", C.c_int64), ("count", C.c_int64), ("attempt", I64), ("k", I64),
                ("eta", D), ("eta_bar", D), ("eta_next", D), ("num", D), ("cross", D),
                ("accepted", I32), ("phase", I32), ("pcap", C.c_int64), ("pcount", C.c_int64),
                ("pol_k", I64), ("pol_cap", I64), ("pol_primal", I64), ("pol_dual", I64),
                ("pol_gap", D)]


class _Cert(C.Structure):
    _fields_ = [("obj", C.c_double), ("res", C.c_double), ("ok", C.c_int32)]


class _KKT(C.Structure):
    _fields_ = [("primal_obj", C.c_double), ("dual_obj", C.c_double), ("rel_gap", C.c_double),
                ("primal_res_abs", C.c_double), ("primal_res_rel", C.c_double),
                ("dual_res_abs", C.c_double), ("dual_res_rel", C.c_double)]


_libs = {}
_threaded = False


def set_threaded(on: bool) -> None:
    """Route later oracle calls to the OpenMP build (all-cores CPU baseline) or
    back to the plain build."""
    global _threaded
    _threaded = bool(on)


def lib():
    key = _threaded
    if key not in _libs:
        _libs[key] = _load(build(threaded=key))
    return _libs[key]


def _load(path):
    if True:
        L = C.CDLL(path)
        L.orc_spmv.argtypes = [C.POINTER(_LP), D, D]
        L.orc_spmv_t.argtypes = [C.POINTER(_LP), D, D]
        L.orc_precondition.argtypes = [C.c_int32, C.c_int32, I32, I32, D, C.c_int32, C.c_int32, D, D]
        L.orc_scale_vectors.argtypes = [C.c_int32, C.c_int32, D, D, D, D, D, D, D, D, D, D, D, D]
        L.orc_initial_primal_weight.argtypes = [C.POINTER(_LP)]
        L.orc_initial_primal_weight.restype = C.c_double
        L.orc_init_state.argtypes = [C.POINTER(_LP), C.POINTER(_State)]
        L.orc_dual_case.argtypes = [C.c_double] * 4
        L.orc_dual_case.restype = C.c_double
        L.orc_adaptive_step.argtypes = [C.POINTER(_LP), C.POINTER(_Params), C.POINTER(_State),
                                        C.POINTER(_Scratch)]
        L.orc_norm_gap.argtypes = [C.POINTER(_LP), D, D, D, D, D, D, C.c_double, D, D]
        L.orc_norm_gap.restype = C.c_double
        L.orc_norm_gap_bisect.argtypes = [C.POINTER(_LP), D, D, D, D, D, D, C.c_double, D]
        L.orc_norm_gap_bisect.restype = C.c_double
        L.orc_path_value.argtypes = [C.POINTER(_LP), D, D, D, D, C.c_double, C.c_double,
                                     C.c_int32, D, D, D]
        L.orc_path_value.restype = C.c_double
        L.orc_primal_weight_update.argtypes = [C.c_double] * 5
        L.orc_primal_weight_update.restype = C.c_double
        L.orc_kkt_eval.argtypes = [C.POINTER(_Unscale), D, D, C.c_int32, D, D, D, D, D,
                                   C.POINTER(_KKT)]
        L.orc_primal_infeas_test.argtypes = [C.POINTER(_Unscale), D, C.c_double, D, D, D,
                                             C.POINTER(_Cert)]
        L.orc_primal_infeas_test.restype = None
        L.orc_dual_infeas_test.argtypes = [C.POINTER(_Unscale), D, C.c_double, D, D,
                                           C.POINTER(_Cert)]
        L.orc_dual_infeas_test.restype = None
        L.orc_pdlp.argtypes = [C.POINTER(_LP), C.POINTER(_Unscale), C.POINTER(_Params),
                               C.POINTER(_State), C.POINTER(_Scratch), D, D, C.POINTER(_Result)]
        L.orc_pdlp.restype = C.c_int32
        L.orc_pdlp_record.argtypes = [C.POINTER(_LP), C.POINTER(_Unscale), C.POINTER(_Params),
                                      C.POINTER(_State), C.POINTER(_Scratch), D, D,
                                      C.POINTER(_Result), C.POINTER(_Tape)]
        L.orc_pdlp_record.restype = C.c_int32
        L.orc_pdlp_trace.argtypes = [C.POINTER(_LP), C.POINTER(_Unscale), C.POINTER(_Params),
                                     C.POINTER(_State), C.POINTER(_Scratch), D, D,
                                     C.POINTER(_Result), C.POINTER(_Tape), C.POINTER(_Trace)]
        L.orc_pdlp_trace.restype = C.c_int32
        L.orc_unroll_replay.argtypes = [C.POINTER(_LP), C.POINTER(_Tape), C.c_int64, D, D, D, D,
                                        C.POINTER(C.c_int64)]
        L.orc_unroll_replay.restype = None
        L.orc_unroll_adjoint.argtypes = [C.POINTER(_LP), C.POINTER(_Tape), C.c_int64, D, D, D, D,
                                         D]
        L.orc_unroll_adjoint.restype = C.c_int32
        L.orc_unroll_tangent.argtypes = [C.POINTER(_LP), C.POINTER(_Tape), C.c_int64, D, D, D, D,
                                         D]
        L.orc_unroll_tangent.restype = C.c_int32
    return L


def _d(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(D)


def _i(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(I32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class LPView:
    """Keeps numpy arrays alive behind an ``orc_lp`` struct."""

    def __init__(self, m, n, row_ptr, col, val, c, lc, uc, lv, uv):
        self.m, self.n = int(m), int(n)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = _f64(val)
        self.c, self.lc, self.uc, self.lv, self.uv = map(_f64, (c, lc, uc, lv, uv))
        self.s = _LP(self.m, self.n, _i(self.row_ptr), _i(self.col), _d(self.val), _d(self.c),
                     _d(self.lc), _d(self.uc), _d(self.lv), _d(self.uv))

    @classmethod
    def of(cls, lp):
        return cls(lp.m, lp.n, lp.row_ptr, lp.col, lp.val, lp.c, lp.lc, lp.uc, lp.lv, lp.uv)

    def ref(self):
        return C.byref(self.s)


def spmv(view: LPView, x) -> np.ndarray:
    x = _f64(x)
    out = np.empty(view.m)
    lib().orc_spmv(view.ref(), _d(x), _d(out))
    return out


def spmv_t(view: LPView, y) -> np.ndarray:
    y = _f64(y)
    out = np.empty(view.n)
    lib().orc_spmv_t(view.ref(), _d(y), _d(out))
    return out


def precondition(lp, ruiz_iters: int = 10, pc: bool = True):
    """Returns (scaled values, d1, d2)."""
    val = np.array(lp.val, dtype=np.float64, copy=True)
    d1 = np.empty(lp.m)
    d2 = np.empty(lp.n)
    rp = np.ascontiguousarray(lp.row_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(lp.col, dtype=np.int32)
    lib().orc_precondition(lp.m, lp.n, _i(rp), _i(cl), _d(val), int(ruiz_iters), int(pc),
                           _d(d1), _d(d2))
    return val, d1, d2


def scale_vectors(lp, d1, d2):
    m, n = lp.m, lp.n
    outs = [np.empty(n), np.empty(m), np.empty(m), np.empty(n), np.empty(n)]
    ins = [_f64(a) for a in (d1, d2, lp.c, lp.lc, lp.uc, lp.lv, lp.uv)]
    lib().orc_scale_vectors(m, n, *[_d(a) for a in ins], *[_d(a) for a in outs])
    return outs  # c, lc, uc, lv, uv


def dual_case(yhat, sigma, lc, uc) -> float:
    return lib().orc_dual_case(float(yhat), float(sigma), float(lc), float(uc))


@dataclasses.dataclass
class Params:
    eps_feas: float = 1e-8
    eps_gap: float = 1e-8
    max_iters: int = 100_000
    check_every: int = 64
    terminate: bool = True
    beta_suff: float = 0.1
    beta_nec: float = 0.9
    beta_art: float = 0.5
    theta: float = 0.5
    eps_zero: float = 1e-10
    red_exp: float = 0.3
    grow_exp: float = 0.6
    reduced_cost_mode: int | None = None   # None: 0 with polishing, 1 without
    polish: bool = False
    polish_first: int = 100
    fixed_step: bool = False
    fixed_eta: float = 0.0
    adaptive_restarts: bool = True
    ruiz_iters: int = 10
    pc: bool = True
    detect_infeasibility: bool = True
    eps_infeas: float = 1e-9
    restart_period: int = 0        # > 0: Algorithm 5 mode (needs fixed_step, fixed_eta)
    fixed_omega: float = 1.0
    signed_step_rule: bool = False  # the printed signed step test (tests only)

    def cstruct(self) -> _Params:
        rc = self.reduced_cost_mode
        if rc is None:
            rc = 0 if self.polish else 1
        return _Params(self.eps_feas, self.eps_gap, int(self.max_iters), int(self.check_every),
                       int(bool(self.terminate)), self.beta_suff, self.beta_nec, self.beta_art,
                       self.theta, self.eps_zero, self.red_exp, self.grow_exp, int(rc),
                       int(bool(self.polish)), int(self.polish_first), int(bool(self.fixed_step)),
                       float(self.fixed_eta), int(bool(self.adaptive_restarts)),
                       int(bool(self.detect_infeasibility)), float(self.eps_infeas),
                       int(self.restart_period), float(self.fixed_omega),
                       int(bool(self.signed_step_rule)))


STATUS = {0: "OPTIMAL", 1: "ITERATION_LIMIT", 3: "NUMERICAL_ERROR", 4: "PRIMAL_INFEASIBLE",
          5: "DUAL_INFEASIBLE"}


def _unit_unscale(view: "LPView"):
    ones = (np.ones(max(view.m, 1)), np.ones(max(view.n, 1)))
    return _Unscale(view.s, _d(ones[0]), _d(ones[1]), 0.0), ones


def primal_infeas_test(lp, y, eps: float = 1e-9) -> dict:
    """Appendix D primal-infeasibility test of y (original units, no scaling).

    Returns obj, res, ok and the projected y, A^T y and r.
    """
    view = LPView.of(lp)
    u, keep = _unit_unscale(view)
    yo, atyo, ro = np.empty(lp.m), np.empty(lp.n), np.empty(lp.n)
    ct = _Cert()
    lib().orc_primal_infeas_test(C.byref(u), _d(_f64(y)), float(eps), _d(yo), _d(atyo), _d(ro),
                                 C.byref(ct))
    return dict(obj=ct.obj, res=ct.res, ok=bool(ct.ok), y=yo, aty=atyo, r=ro)


def dual_infeas_test(lp, x, eps: float = 1e-9) -> dict:
    """Appendix D dual-infeasibility test of x (original units, no scaling).

    Returns obj, res, ok and the projected x and A x.
    """
    view = LPView.of(lp)
    u, keep = _unit_unscale(view)
    xo, axo = np.empty(lp.n), np.empty(lp.m)
    ct = _Cert()
    lib().orc_dual_infeas_test(C.byref(u), _d(_f64(x)), float(eps), _d(xo), _d(axo), C.byref(ct))
    return dict(obj=ct.obj, res=ct.res, ok=bool(ct.ok), x=xo, ax=axo)


class Solver:
    """Oracle PDLP on one LP: preconditions, initializes, iterates or solves.

    All quantities exposed here are in the scaled space except the results
    of :meth:`kkt` and the unscaled solution returned by :meth:`solution`.
    """

    def __init__(self, lp, params: Params | None = None, scale: bool = True, precond=None):
        self.lp = lp
        self.params = params or Params()
        m, n = lp.m, lp.n
        self.m, self.n = m, n
        if precond is not None:      # (val, d1, d2) of an earlier precondition(lp, ...)
            val, d1, d2 = precond
        elif scale:
            val, d1, d2 = precondition(lp, self.params.ruiz_iters, self.params.pc)
        else:
            val, d1, d2 = np.array(lp.val, dtype=np.float64), np.ones(m), np.ones(n)
        self.d1, self.d2 = d1, d2
        cs, lcs, ucs, lvs, uvs = scale_vectors(lp, d1, d2)
        self.scaled = LPView(m, n, lp.row_ptr, lp.col, val, cs, lcs, ucs, lvs, uvs)
        self.orig = LPView.of(lp)
        self.uns = _Unscale(self.orig.s, _d(self.d1), _d(self.d2), float(lp.obj_offset))
        z = lambda k: np.zeros(k)
        self.arr = {k: z(n) for k in ("x", "aty", "x0", "sx")}
        self.arr.update({k: z(m) for k in ("y", "ax", "y0", "sy")})
        self.st = _State(*[_d(self.arr[k]) for k in ("x", "y", "ax", "aty", "x0", "y0", "sx", "sy")])
        self.scr_arr = [z(max(n, 1)) for _ in range(6)] + [z(max(m, 1)) for _ in range(6)]
        self.scr = _Scratch(*[_d(a) for a in self.scr_arr])
        lib().orc_init_state(self.scaled.ref(), C.byref(self.st))
        self.out_x = z(n)
        self.out_y = z(m)
        self.result = None

    # -- state access
    def __getattr__(self, name):
        arr = self.__dict__.get("arr")
        if arr is not None and name in arr:
            return arr[name]
        raise AttributeError(name)

    @property
    def omega(self):
        return self.st.omega

    @property
    def eta_hat(self):
        return self.st.eta_hat

    @property
    def k(self):
        return self.st.k

    def counters(self) -> dict:
        s = self.st
        return dict(k=s.k, t=s.t, n_outer=s.n_outer, attempts=s.attempts, kkt_passes=s.kkt_passes,
                    restarts_i=s.restarts_i, restarts_ii=s.restarts_ii, restarts_iii=s.restarts_iii,
                    omega=s.omega, eta_hat=s.eta_hat, seta=s.seta, mu_ref=s.mu_ref,
                    mu_c_prev=s.mu_c_prev, last_eta=s.last_eta, last_eta_bar=s.last_eta_bar)

    # -- running
    def _run(self, params: Params) -> dict:
        res = _Result()
        cp = params.cstruct()
        lib().orc_pdlp(self.scaled.ref(), C.byref(self.uns), C.byref(cp), C.byref(self.st),
                       C.byref(self.scr), _d(self.out_x), _d(self.out_y), C.byref(res))
        d = {f: getattr(res, f) for f, _ in _Result._fields_}
        d["status_name"] = STATUS.get(d["status"], str(d["status"]))
        self.result = d
        return d

    def traced(self, params: Params | None = None, cap: int = 1 << 16,
               pcap: int = 64) -> dict:
        """Run with `params` (default: this solver's) recording every step
        attempt and polishing point (see orc_trace).  Returns the result dict
        with the trace arrays under "trace" (first min(count, cap) entries)."""
        params = params or self.params
        a = {k: np.zeros(cap, dtype=np.int64) for k in ("attempt", "k")}
        a.update({k: np.zeros(cap) for k in ("eta", "eta_bar", "eta_next", "num", "cross")})
        a.update({k: np.zeros(cap, dtype=np.int32) for k in ("accepted", "phase")})
        pa = {k: np.zeros(pcap, dtype=np.int64) for k in ("pol_k", "pol_cap", "pol_primal",
                                                          "pol_dual")}
        pa["pol_gap"] = np.zeros(pcap)
        ptr = lambda v: v.ctypes.data_as(I64 if v.dtype == np.int64 else
                                         (I32 if v.dtype == np.int32 else D))
        tr = _Trace(cap, 0, *[ptr(a[k]) for k in ("attempt", "k", "eta", "eta_bar", "eta_next",
                                                  "num", "cross", "accepted", "phase")],
                    pcap, 0, *[ptr(pa[k]) for k in ("pol_k", "pol_cap", "pol_primal",
                                                    "pol_dual", "pol_gap")])
        res = _Result()
        cp = params.cstruct()
        lib().orc_pdlp_trace(self.scaled.ref(), C.byref(self.uns), C.byref(cp),
                             C.byref(self.st), C.byref(self.scr), _d(self.out_x),
                             _d(self.out_y), C.byref(res), None, C.byref(tr))
        d = {f: getattr(res, f) for f, _ in _Result._fields_}
        d["status_name"] = STATUS.get(d["status"], str(d["status"]))
        nt, npol = min(tr.count, cap), min(tr.pcount, pcap)
        t = {k: v[:nt].copy() for k, v in a.items()}
        t.update({k: v[:npol].copy() for k, v in pa.items()})
        t["count"], t["pcount"] = tr.count, tr.pcount
        d["trace"] = t
        self.result = d
        return d

    def iterate(self, k: int) -> dict:
        """Exactly k more accepted steps, restart checks on, no termination."""
        p = dataclasses.replace(self.params, terminate=False, max_iters=self.st.k + int(k),
                                polish=False)
        return self._run(p)

    def step(self) -> None:
        """One bare adaptive PDHG step (Algorithm 2) without averaging or checks."""
        cp = self.params.cstruct()
        rc = lib().orc_adaptive_step(self.scaled.ref(), C.byref(cp), C.byref(self.st),
                                     C.byref(self.scr))
        if rc != 0:
            raise FloatingPointError("numerical error in PDHG step")

    def solve(self) -> dict:
        return self._run(self.params)

    def solution(self):
        """Unscaled (x, y) of the returned point: x = D2 x~, y = D1 y~."""
        return self.d2 * self.out_x, self.d1 * self.out_y

    def kkt(self, xs, ys, mode: int | None = None) -> dict:
        if mode is None:
            mode = 0 if self.params.polish else 1
        k = _KKT()
        sc = [np.empty(self.n) for _ in range(3)] + [np.empty(self.m) for _ in range(2)]
        lib().orc_kkt_eval(C.byref(self.uns), _d(_f64(xs)), _d(_f64(ys)), int(mode),
                           *[_d(a) for a in sc], C.byref(k))
        return {f: getattr(k, f) for f, _ in _KKT._fields_}

    def gap(self, x, y, ax, aty, xr, yr, omega, bisect=False) -> float:
        return norm_gap(self.scaled, x, y, ax, aty, xr, yr, omega, bisect)


def norm_gap(view: LPView, x, y, ax, aty, xr, yr, omega, bisect=False) -> float:
    x, y, ax, aty, xr, yr = map(_f64, (x, y, ax, aty, xr, yr))
    g = np.empty(max(view.n, 1))
    if bisect:
        return lib().orc_norm_gap_bisect(view.ref(), _d(x), _d(y), _d(ax), _d(aty), _d(xr),
                                         _d(yr), float(omega), _d(g))
    bp = np.empty(2 * (view.m + view.n) + 1)
    return lib().orc_norm_gap(view.ref(), _d(x), _d(y), _d(ax), _d(aty), _d(xr), _d(yr),
                              float(omega), _d(g), _d(bp))


def path_value(view: LPView, x, y, ax, aty, omega, s, which):
    """D(s) (which=0) or f(z^(s)) (which=1) on the proximal path; also returns z^(s)."""
    x, y, ax, aty = map(_f64, (x, y, ax, aty))
    g = np.empty(max(view.n, 1))
    xh = np.empty(view.n)
    yh = np.empty(view.m)
    v = lib().orc_path_value(view.ref(), _d(x), _d(y), _d(ax), _d(aty), float(omega), float(s),
                             int(which), _d(g), _d(xh), _d(yh))
    return v, xh, yh


def primal_weight_update(dx, dy, omega, theta=0.5, eps_zero=1e-10) -> float:
    return lib().orc_primal_weight_update(float(dx), float(dy), float(omega), float(theta),
                                          float(eps_zero))


def initial_primal_weight(view: LPView) -> float:
    return lib().orc_initial_primal_weight(view.ref())


def scale_by(lp, d1, d2, c=None, lc=None, uc=None, val=None):
    """Scaled data of `lp` (or of replacement c, lc, uc, val in original units)
    under fixed diagonals: A~ = D1 A D2 entry by entry as (d1_i a_ij) d2_j,
    c~ = D2 c, (lc~, uc~) = D1 (lc, uc), (lv~, uv~) = (lv, uv) / D2."""
    m, n = lp.m, lp.n
    rp = np.asarray(lp.row_ptr, dtype=np.int64)
    rows = np.repeat(np.arange(m), np.diff(rp))
    cols = np.asarray(lp.col, dtype=np.int64)
    val = np.asarray(lp.val if val is None else val, dtype=np.float64)
    vs = (d1[rows] * val) * d2[cols]
    cc = lp.c if c is None else c
    l = lp.lc if lc is None else lc
    u = lp.uc if uc is None else uc
    fake = type("_D", (), {})()
    fake.m, fake.n, fake.c, fake.lc, fake.uc, fake.lv, fake.uv = m, n, cc, l, u, lp.lv, lp.uv
    cs, lcs, ucs, lvs, uvs = scale_vectors(fake, d1, d2)
    return LPView(m, n, lp.row_ptr, lp.col, vs, cs, lcs, ucs, lvs, uvs)


class Unroll:
    """K accepted steps of Algorithm 1 with their decisions recorded, and the
    map they define with those decisions held fixed (pdlp_oracle_unroll.c).

    Scaling: D1, D2 from the preconditioning of `lp`; every scaled quantity is
    formed from the original data by scale_by, for the recorded run and for
    replays of perturbed data alike.  Gradients are returned in original
    units: dc = D2 dc~, dlc = D1 dlc~ (0 where lc is infinite), likewise uc,
    dA_ij = D1_i D2_j dA~_ij; the upstream gradient on x = D2 x~ enters as
    D2 dL/dx.
    """

    def __init__(self, lp, K: int, params: Params | None = None):
        self.lp, self.K = lp, int(K)
        prm = dataclasses.replace(params or Params(), terminate=False, max_iters=int(K),
                                  polish=False)
        _, self.d1, self.d2 = precondition(lp, prm.ruiz_iters, prm.pc)
        self.view = scale_by(lp, self.d1, self.d2)
        m, n = lp.m, lp.n
        z = lambda k: np.zeros(k)
        arr = {k: z(n) for k in ("x", "aty", "x0", "sx")}
        arr.update({k: z(m) for k in ("y", "ax", "y0", "sy")})
        st = _State(*[_d(arr[k]) for k in ("x", "y", "ax", "aty", "x0", "y0", "sx", "sy")])
        scr_arr = [z(max(n, 1)) for _ in range(6)] + [z(max(m, 1)) for _ in range(6)]
        scr = _Scratch(*[_d(a) for a in scr_arr])
        lib().orc_init_state(self.view.ref(), C.byref(st))
        self.eta = np.zeros(max(self.K, 1))
        self.omega = np.zeros(max(self.K, 1))
        self.restart = np.zeros(max(self.K, 1), dtype=np.int32)
        self.tape = _Tape(self.K, _d(self.eta), _d(self.omega), _i(self.restart))
        orig = LPView.of(lp)
        uns = _Unscale(orig.s, _d(self.d1), _d(self.d2), 0.0)
        ox, oy = z(n), z(m)
        res = _Result()
        lib().orc_pdlp_record(self.view.ref(), C.byref(uns), C.byref(prm.cstruct()), C.byref(st),
                              C.byref(scr), _d(ox), _d(oy), C.byref(res), C.byref(self.tape))
        self.result = {f: getattr(res, f) for f, _ in _Result._fields_}
        self.x_scaled = arr["x"].copy()
        self.x = self.d2 * self.x_scaled

    def replay(self, c=None, lc=None, uc=None, val=None):
        """x_K (original units) and the activity signature for the given data."""
        view = self.view if all(a is None for a in (c, lc, uc, val)) else \
            scale_by(self.lp, self.d1, self.d2, c, lc, uc, val)
        x = np.zeros(self.lp.n)
        sig = C.c_int64()
        lib().orc_unroll_replay(view.ref(), C.byref(self.tape), self.K, _d(x), None, None, None,
                                C.byref(sig))
        return self.d2 * x, sig.value

    def tangent(self, dc=None, dlc=None, duc=None, dval=None) -> np.ndarray:
        """Directional derivative of x_K (original units) along a direction of
        the data in original units (None = zero): the scaled direction is
        dc~ = D2 dc, dlc~ = D1 dlc, duc~ = D1 duc (0 where the bound is
        infinite), dA~_ij = D1_i D2_j dA_ij; the result is D2 dx~_K."""
        lp = self.lp
        m, n = lp.m, lp.n
        nnz = int(np.asarray(lp.row_ptr)[-1]) if m else 0
        z = lambda k, a: np.zeros(k) if a is None else _f64(a)
        dc, dlc, duc, dval = z(n, dc), z(m, dlc), z(m, duc), z(nnz, dval)
        fin_l = np.isfinite(np.asarray(lp.lc, dtype=np.float64))
        fin_u = np.isfinite(np.asarray(lp.uc, dtype=np.float64))
        rp = np.asarray(lp.row_ptr, dtype=np.int64)
        rows = np.repeat(np.arange(m), np.diff(rp))
        cols = np.asarray(lp.col, dtype=np.int64)
        sdc = _f64(self.d2 * dc)
        sdl = _f64(np.where(fin_l, self.d1 * dlc, 0.0))
        sdu = _f64(np.where(fin_u, self.d1 * duc, 0.0))
        sdv = _f64(self.d1[rows] * self.d2[cols] * dval)
        dx = np.zeros(n)
        rc = lib().orc_unroll_tangent(self.view.ref(), C.byref(self.tape), self.K, _d(sdc),
                                      _d(sdl), _d(sdu), _d(sdv) if sdv.size else None, _d(dx))
        if rc != 0:
            raise MemoryError("oracle tangent out of memory")
        return self.d2 * dx

    def backward(self, gx) -> dict:
        """Gradients of <gx, x_K> in original units (dc, dlc, duc, dval)."""
        lp = self.lp
        m, n = lp.m, lp.n
        gxs = _f64(self.d2 * np.asarray(gx, dtype=np.float64))
        gc, glc, guc = np.zeros(n), np.zeros(m), np.zeros(m)
        gval = np.zeros(int(np.asarray(lp.row_ptr)[-1]) if m else 0)
        rc = lib().orc_unroll_adjoint(self.view.ref(), C.byref(self.tape), self.K, _d(gxs),
                                      _d(gc), _d(glc), _d(guc), _d(gval) if gval.size else None)
        if rc != 0:
            raise MemoryError("oracle adjoint out of memory")
        rp = np.asarray(lp.row_ptr, dtype=np.int64)
        rows = np.repeat(np.arange(m), np.diff(rp))
        cols = np.asarray(lp.col, dtype=np.int64)
        fin_l = np.isfinite(np.asarray(lp.lc, dtype=np.float64))
        fin_u = np.isfinite(np.asarray(lp.uc, dtype=np.float64))
        return {"c": self.d2 * gc, "lc": np.where(fin_l, self.d1 * glc, 0.0),
                "uc": np.where(fin_u, self.d1 * guc, 0.0),
                "val": self.d1[rows] * self.d2[cols] * gval}
