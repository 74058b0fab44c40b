"""pdlp_spmv_noalloc (products staged in a fixed device array, no allocation)
against pdlp_spmv on the same problems, through the C ABI.

Two calls in a row, the second on a smaller problem; both transposes, scaled
and original units; the two-phase A^T y' product and the one-pass one.  The
same kernels run in the same order, so results are bitwise those of
pdlp_spmv.  A problem with m + n above the staging capacity is refused."""
import ctypes as C

import numpy as np
import pytest

import lpgen
import paper_2501_07018_amd as pd

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", flush=True)


class _Dev:
    def __init__(self):
        pd.lib()
        self.hip = C.CDLL("libamdhip64.so.7")
        self.hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        self.hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        self.hip.hipFree.argtypes = [C.c_void_p]
        self.ptrs = []

    def alloc(self, nbytes):
        p = C.c_void_p()
        assert self.hip.hipMalloc(C.byref(p), max(nbytes, 8)) == 0
        self.ptrs.append(p)
        return p.value

    def put(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        p = self.alloc(a.nbytes)
        if a.nbytes:
            assert self.hip.hipMemcpy(p, a.ctypes.data, a.nbytes, 1) == 0
        return p

    def get(self, p, n):
        out = np.empty(n)
        assert self.hip.hipDeviceSynchronize() == 0
        if n:
            assert self.hip.hipMemcpy(out.ctypes.data, p, out.nbytes, 2) == 0
        return out

    def close(self):
        for p in self.ptrs:
            self.hip.hipFree(p)
        self.ptrs = []


def _check_problem(dev, lp, params):
    prob = pd.Problem(lp, params)
    rng = np.random.default_rng(lp.m + 7 * lp.n)
    for transpose in (0, 1):
        n_in, n_out = (lp.m, lp.n) if transpose else (lp.n, lp.m)
        x = rng.standard_normal(n_in)
        for scaled in (1, 0):
            want, _ = prob.spmv(x, transpose=bool(transpose), scaled=bool(scaled))
            xd, od = dev.put(x), dev.alloc(8 * n_out)
            pd.pdlp_spmv_noalloc(prob.h, xd, od, transpose=transpose, scaled=scaled)
            got = dev.get(od, n_out)
            assert np.array_equal(got, want), (lp.m, lp.n, transpose, scaled)
    prob.close()


def test_noalloc_products_match_pdlp_spmv():
    dev = _Dev()
    try:
        say("no-alloc product: 30000 x 40000 skewed LP, two-phase A^T y'")
        _check_problem(dev, lpgen.planted_skewed(30000, 40000, seed=3, n_dense=40),
                       pd.pdlp_params_default(segmented_gathers=1))
        say("no-alloc product: second call on a smaller LP (1000 x 2000, one-pass)")
        _check_problem(dev, lpgen.small_lp(), pd.pdlp_params_default(segmented_gathers=0))
    finally:
        dev.close()


def test_noalloc_refuses_problems_beyond_its_capacity():
    say("no-alloc product: m + n beyond the staging capacity")
    k = (1 << 22) + 1                     # m + n = 2^23 + 2
    lp = lpgen.LP(k, k, np.arange(k + 1, dtype=np.int32), np.arange(k, dtype=np.int32),
                  np.ones(k), np.zeros(k), np.zeros(k), np.ones(k), np.zeros(k), np.ones(k))
    dev = _Dev()
    try:
        prob = pd.Problem(lp, pd.pdlp_params_default(segmented_gathers=0))
        xd, od = dev.put(np.ones(k)), dev.alloc(8 * k)
        with pytest.raises(pd.PdlpError) as ei:
            pd.pdlp_spmv_noalloc(prob.h, xd, od)
        assert ei.value.code == pd.PDLP_ERR_INVALID_ARGUMENT
        prob.close()
        # the entry point still works afterwards
        _check_problem(dev, lpgen.small_lp(1), pd.pdlp_params_default())
    finally:
        dev.close()
