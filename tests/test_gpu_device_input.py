"""pdlp_problem_create_device: the same problem as pdlp_problem_create when
the arrays live in GPU memory.

The arrays are placed on the device with the HIP runtime the library itself
uses (hipMalloc/hipMemcpy through ctypes), and, in a child process, as torch
tensors through Problem.from_tensors.  Both must give bitwise the same
preconditioned problem and the same solve as the host-array call.
"""
import ctypes as C
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import lpgen
import paper_2501_07018_amd as pd
from tests.test_gpu_parity import gpu_params, say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


class _DeviceArrays:
    """Device copies of host arrays, freed on close."""

    def __init__(self):
        pd.lib()  # the library's HIP runtime is the one already loaded
        self.hip = C.CDLL("libamdhip64.so.7")
        self.hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        self.hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        self.hip.hipFree.argtypes = [C.c_void_p]
        self.ptrs = []

    def put(self, a):
        a = np.ascontiguousarray(a)
        p = C.c_void_p()
        assert self.hip.hipMalloc(C.byref(p), max(a.nbytes, 8)) == 0
        self.ptrs.append(p)
        if a.nbytes:
            assert self.hip.hipMemcpy(p, a.ctypes.data, a.nbytes, 1) == 0  # host to device
        return p.value

    def close(self):
        for p in self.ptrs:
            self.hip.hipFree(p)
        self.ptrs = []


def _create_device(lp, dev, params=None):
    arrs = [np.asarray(lp.row_ptr, np.int32), np.asarray(lp.col, np.int32)] + \
           [np.asarray(getattr(lp, k), np.float64) for k in ("val", "c", "lc", "uc", "lv", "uv")]
    h = pd.pdlp_problem_create_device(lp.m, lp.n, lp.nnz, *[dev.put(a) for a in arrs],
                                      0.0, params, None)
    p = pd.Problem.__new__(pd.Problem)
    p.m, p.n, p.h = lp.m, lp.n, h
    return p


def test_device_arrays_give_the_host_problem():
    say("create from device arrays")
    dev = _DeviceArrays()
    try:
        for lp in (lpgen.small_lp(), lpgen.planted_skewed(3000, 5000, seed=103, n_dense=3)):
            host = pd.Problem(lp)
            devp = _create_device(lp, dev)
            gh, gd = host.scaled(), devp.scaled()
            for k in gh:
                assert np.array_equal(gh[k], gd[k]), k
            prm = gpu_params(eps_feas=1e-6, eps_gap=1e-6, max_iters=20000)
            rh, rd = host.solve(prm), devp.solve(prm)
            assert rh["status_name"] == rd["status_name"] and rh["iterations"] == rd["iterations"]
            for k in ("x", "y", "r"):
                assert np.array_equal(rh[k], rd[k]), k
            host.close()
            devp.close()
        # validation applies to device input as to host input
        bad = lpgen.small_lp()
        bad.lc = bad.lc.copy()
        bad.lc[0] = bad.uc[0] + 1.0
        with pytest.raises(pd.PdlpError) as ei:
            _create_device(bad, dev)
        assert ei.value.code == pd.PDLP_ERR_INVALID_ARGUMENT
    finally:
        dev.close()


_CHILD = r"""
import json, sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
import lpgen
import paper_2501_07018_amd as pd
lp = lpgen.small_lp()
d = torch.device("cuda:0")
t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dtype=dt, device=d)
i32, f64 = torch.int32, torch.float64
p = pd.Problem.from_tensors(lp.m, lp.n, t(lp.row_ptr, i32), t(lp.col, i32), t(lp.val, f64),
                            t(lp.c, f64), t(lp.lc, f64), t(lp.uc, f64), t(lp.lv, f64),
                            t(lp.uv, f64))
r = p.solve(pd.pdlp_params_default(eps_feas=1e-6, eps_gap=1e-6, max_iters=20000))
# tensors of the wrong length are refused before anything is copied
short = []
for k in ("row_ptr", "col", "val", "c", "lc", "uc", "lv", "uv"):
    a = {kk: np.asarray(getattr(lp, kk)) for kk in ("row_ptr", "col", "val", "c", "lc", "uc",
                                                    "lv", "uv")}
    a[k] = a[k][:-1]
    ts = [t(a["row_ptr"], i32), t(a["col"], i32)] + [t(a[kk], f64) for kk in
                                                   ("val", "c", "lc", "uc", "lv", "uv")]
    try:
        pd.Problem.from_tensors(lp.m, lp.n, *ts)
        short.append((k, "accepted"))
    except ValueError:
        short.append((k, "refused"))
print(json.dumps({"status": r["status_name"], "iterations": r["iterations"],
                  "x": r["x"].tolist(), "short": short}))
"""


def test_torch_tensors_give_the_host_problem():
    say("create from torch tensors (child process)")
    pytest.importorskip("torch")
    out = subprocess.run([sys.executable, "-c", _CHILD, ROOT], capture_output=True, text=True,
                         timeout=240)
    assert out.returncode == 0, out.stderr[-2000:]
    got = json.loads(out.stdout.strip().splitlines()[-1])
    r = pd.Problem(lpgen.small_lp()).solve(pd.pdlp_params_default(eps_feas=1e-6, eps_gap=1e-6,
                                                                  max_iters=20000))
    assert got["status"] == r["status_name"] and got["iterations"] == r["iterations"]
    assert np.array_equal(np.array(got["x"]), r["x"])
    assert got["short"] and all(v == "refused" for _, v in got["short"]), got["short"]


_LAYER_CHILD = r"""
import json, sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
import lpgen
import paper_2501_07018_amd as pd
from paper_2501_07018_amd.layer import LPLayer
lps = [lpgen.planted_uniform(60, 100, 5, seed=3), lpgen.planted_uniform(150, 225, 8, seed=101)]
cat = lambda k: np.concatenate([np.asarray(getattr(lp, k), dtype=np.float64) for lp in lps])
gx = np.random.default_rng(3).standard_normal(sum(lp.n for lp in lps))
out = {}
for where in ("cpu", "cuda"):
    layer = LPLayer(lps, K=60, ckpt=25)
    ts = [torch.tensor(cat(k), device=where, requires_grad=True) for k in ("c", "lc", "uc", "val")]
    x = layer(*ts)
    (x * torch.tensor(gx, device=where)).sum().backward()
    out[where] = [x.detach().cpu().numpy()] + [t.grad.detach().cpu().numpy() for t in ts]
    out[where + "_device"] = str(x.device)
same = [bool(np.array_equal(a, b)) for a, b in zip(out["cpu"], out["cuda"])]
# the device variants reject invalid data like the host ones
u = pd.Unroll(lps)
bad = torch.tensor(cat("c"), device="cuda")
bad[3] = float("nan")
try:
    u.set_data_device(c=bad.data_ptr(), stream=torch.cuda.current_stream().cuda_stream)
    refused = False
except pd.PdlpError as e:
    refused = e.code == pd.PDLP_ERR_INVALID_ARGUMENT
print(json.dumps({"same": same, "device": out["cuda_device"], "refused": refused}))
"""


def test_layer_on_device_tensors_matches_the_host_path():
    say("LPLayer on CUDA tensors vs host tensors (child process)")
    pytest.importorskip("torch")
    out = subprocess.run([sys.executable, "-c", _LAYER_CHILD, ROOT], capture_output=True,
                         text=True, timeout=240)
    assert out.returncode == 0, out.stderr[-2000:]
    got = json.loads(out.stdout.strip().splitlines()[-1])
    assert got["device"].startswith("cuda"), got
    assert all(got["same"]), got    # x_K and the four gradients, bitwise
    assert got["refused"], got


_BATCH_CHILD = r"""
import json, sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
import lpgen
import paper_2501_07018_amd as pd
from paper_2501_07018_amd.layer import LPLayer
lps = [lpgen.planted_uniform(150, 225, 8, seed=101), lpgen.tiny_random_lp(104, 7, 12),
       lpgen.planted_skewed(1000, 2000, seed=106, mean_degree=4.0, cap=500, n_dense=10,
                            dense_frac=0.3)]
d = torch.device("cuda:0")
i32, f64 = torch.int32, torch.float64
keys = ("row_ptr", "col", "val", "c", "lc", "uc", "lv", "uv")
def cat(k, lst=lps):
    return np.concatenate([np.asarray(getattr(lp, k)) for lp in lst])
def tens(arrs):
    return [torch.as_tensor(np.ascontiguousarray(arrs[k])).to(
        dtype=i32 if k in ("row_ptr", "col") else f64, device=d) for k in keys]
m = [lp.m for lp in lps]
n = [lp.n for lp in lps]
nnz = [lp.nnz for lp in lps]
arrs = {k: cat(k) for k in keys}
prm = pd.pdlp_params_default(eps_feas=1e-7, eps_gap=1e-7, max_iters=6000)
rh = pd.Batch(lps).solve(prm)
rd = pd.Batch.from_tensors(m, n, nnz, *tens(arrs)).solve(prm)
batch_same = all(a["status_name"] == b["status_name"] and a["iterations"] == b["iterations"]
                 and all(np.array_equal(a[k], b[k]) for k in ("x", "y", "r"))
                 for a, b in zip(rh, rd))
# wrong lengths are refused before anything is handed over
short = []
for k in keys:
    a = dict(arrs)
    a[k] = a[k][:-1]
    try:
        pd.Batch.from_tensors(m, n, nnz, *tens(a))
        short.append((k, "accepted"))
    except ValueError:
        short.append((k, "refused"))
# invalid data in one instance is refused by the library, naming the instance
bad = dict(arrs)
bad["lc"] = arrs["lc"].copy()
bad["lc"][lps[0].m + 1] = bad["uc"][lps[0].m + 1] + 1.0
try:
    pd.Batch.from_tensors(m, n, nnz, *tens(bad))
    invalid = "accepted"
except pd.PdlpError as e:
    invalid = "instance 1" if (e.code == pd.PDLP_ERR_INVALID_ARGUMENT and "instance 1" in str(e)) else str(e)
# the unrolled map and the layer built from device tensors
lay = [lpgen.planted_uniform(60, 100, 5, seed=3), lpgen.planted_uniform(150, 225, 8, seed=101)]
la = {k: cat(k, lay) for k in keys}
lm, ln, lz = [lp.m for lp in lay], [lp.n for lp in lay], [lp.nnz for lp in lay]
uh = pd.Unroll(lay)
ud = pd.Unroll.from_tensors(lm, ln, lz, *tens(la))
xh, xd = uh.forward(60, 25), ud.forward(60, 25)
gx = np.random.default_rng(3).standard_normal(len(xh))
gh, gd = uh.backward(gx), ud.backward(gx)
unroll_same = bool(np.array_equal(xh, xd)) and all(np.array_equal(gh[k], gd[k]) for k in gh)
layers = []
for layer in (LPLayer(lay, K=60, ckpt=25), LPLayer.from_tensors(lm, ln, lz, *tens(la), K=60,
                                                                ckpt=25)):
    ts = [torch.tensor(la[k], device=d, requires_grad=True) for k in ("c", "lc", "uc", "val")]
    x = layer(*ts)
    (x * torch.tensor(gx, device=d)).sum().backward()
    layers.append([x.detach().cpu().numpy()] + [t.grad.detach().cpu().numpy() for t in ts])
layer_same = all(np.array_equal(a, b) for a, b in zip(*layers))
print(json.dumps({"batch_same": batch_same, "short": short, "invalid": invalid,
                  "unroll_same": unroll_same, "layer_same": bool(layer_same)}))
"""


def test_batch_and_unroll_from_device_tensors_match_the_host_path():
    say("Batch / Unroll / LPLayer from CUDA tensors vs host arrays (child process)")
    pytest.importorskip("torch")
    out = subprocess.run([sys.executable, "-c", _BATCH_CHILD, ROOT], capture_output=True,
                         text=True, timeout=240)
    assert out.returncode == 0, out.stderr[-2000:]
    got = json.loads(out.stdout.strip().splitlines()[-1])
    assert got["batch_same"], got          # solves bitwise equal to the host-array batch
    assert got["short"] and all(v == "refused" for _, v in got["short"]), got["short"]
    assert got["invalid"] == "instance 1", got
    assert got["unroll_same"], got         # x_K and gradients bitwise equal
    assert got["layer_same"], got
