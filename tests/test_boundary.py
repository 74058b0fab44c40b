"""CPU checks of the C-ABI boundary: the library loads, exports every entry
point declared in include/pdlp.h, its ctypes structs match the C layout, and
input validation rejects bad problems before any GPU work."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2501_07018_amd as pd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdlp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdlp_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = pd.lib()
    names = declared_functions()
    assert "pdlp_solve" in names and "pdlp_iterate_k" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(pd.EXPORTS)


def test_struct_layout_matches_header(tmp_path):
    structs = {"pdlp_params": pd.Params, "pdlp_result": pd.Result,
               "pdlp_iter_info": pd.IterInfo, "pdlp_state_blob": pd.StateBlob,
               "pdlp_kernel_stats": pd.KernelStats, "pdlp_device_rates": pd.DeviceRates,
               "pdlp_batch_stats": pd.BatchStats, "pdlp_unroll_stats": pd.UnrollStats}
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "pdlp.h"', "int main(void){"]
    for cname, py in structs.items():
        src.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            src.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    src.append("return 0;}")
    c_file = tmp_path / "layout.c"
    c_file.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), str(c_file), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, f"{cname}.{f}"


def _tiny():
    return dict(m=2, n=3, row_ptr=np.array([0, 2, 3], np.int32), col=np.array([0, 2, 1], np.int32),
                val=np.array([1.0, 2.0, 3.0]), c=np.ones(3), lc=np.array([0.0, -np.inf]),
                uc=np.array([1.0, 4.0]), lv=np.zeros(3), uv=np.ones(3))


@pytest.mark.parametrize("mutate,msg", [
    (lambda d: d.update(col=np.array([2, 0, 1], np.int32)), "increasing"),
    (lambda d: d.update(col=np.array([0, 0, 1], np.int32)), "increasing"),
    (lambda d: d.update(col=np.array([0, 3, 1], np.int32)), "out of range"),
    (lambda d: d.update(val=np.array([1.0, np.nan, 3.0])), "non-finite"),
    (lambda d: d.update(c=np.array([1.0, np.inf, 0.0])), "non-finite"),
    (lambda d: d.update(lc=np.array([2.0, -np.inf])), "lc > uc"),
    (lambda d: d.update(lv=np.array([0.0, 2.0, 0.0])), "lv > uv"),
    (lambda d: d.update(lc=np.array([np.inf, -np.inf]), uc=np.array([np.inf, 4.0])), "wrong infinity"),
    (lambda d: d.update(uv=np.array([1.0, -np.inf, 1.0]), lv=np.array([0.0, -np.inf, 0.0])), "wrong infinity"),
    (lambda d: d.update(lc=np.array([np.nan, -np.inf])), "NaN"),
    (lambda d: d.update(row_ptr=np.array([0, 3, 2], np.int32)), "nondecreasing"),
    (lambda d: d.update(row_ptr=np.array([1, 2, 3], np.int32)), "row_ptr[0]"),
])
def test_invalid_problems_are_rejected_before_gpu_work(mutate, msg):
    d = _tiny()
    mutate(d)
    with pytest.raises(pd.PdlpError) as ei:
        pd.pdlp_problem_create(d["m"], d["n"], d["row_ptr"], d["col"], d["val"], d["c"], d["lc"],
                               d["uc"], d["lv"], d["uv"])
    assert ei.value.code == pd.PDLP_ERR_INVALID_ARGUMENT
    assert msg in str(ei.value)


def test_params_defaults_are_the_papers_constants():
    p = pd.pdlp_params_default()
    assert p.check_every == 64 and p.ruiz_iters == 10 and p.pock_chambolle == 1
    assert (p.beta_suff, p.beta_nec, p.beta_art) == (0.1, 0.9, 0.5)
    assert (p.theta, p.eps_zero, p.red_exp, p.grow_exp) == (0.5, 1e-10, 0.3, 0.6)
    assert p.polish_first == 100


class _Obj:
    def __init__(self, d):
        self.__dict__.update(d)


@pytest.mark.parametrize("mutate,msg", [
    (lambda d: d.update(col=np.array([0, 3, 1], np.int32)), "out of range"),
    (lambda d: d.update(col=np.array([2, 0, 1], np.int32)), "increasing"),
    (lambda d: d.update(val=np.array([1.0, np.nan, 3.0])), "non-finite"),
    (lambda d: d.update(lc=np.array([2.0, -np.inf])), "lc > uc"),
    (lambda d: d.update(row_ptr=np.array([0, 3, 2], np.int32)), "nondecreasing"),
    (lambda d: d.update(row_ptr=np.array([1, 2, 3], np.int32)), "row_ptr[0]"),
])
def test_invalid_batches_name_the_instance_before_gpu_work(mutate, msg):
    good, bad = _tiny(), _tiny()
    mutate(bad)
    with pytest.raises(pd.PdlpError) as ei:
        pd.pdlp_batch_create([_Obj(good), _Obj(bad), _Obj(_tiny())])
    assert ei.value.code == pd.PDLP_ERR_INVALID_ARGUMENT
    assert "instance 1: " in str(ei.value) and msg in str(ei.value)


def test_empty_batch_is_rejected():
    h = C.c_void_p()
    rc = pd.lib().pdlp_batch_create(0, None, None, None, None, None, None, None, None, None,
                                    None, None, None, None, None, C.byref(h))
    assert rc == pd.PDLP_ERR_INVALID_ARGUMENT and not h.value


@pytest.mark.parametrize("fn", ["pdlp_batch_create_device", "pdlp_unroll_create_device"])
def test_device_batch_creation_checks_sizes_before_any_copy(fn):
    """The device-input creation calls check the host size arrays (and NULL
    data pointers) before they copy anything, so bad sizes never reach the
    runtime; here no GPU is present at all."""
    f = getattr(pd.lib(), fn)
    extra = [None] if fn == "pdlp_batch_create_device" else []   # obj_offset
    h = C.c_void_p()
    rc = f(0, None, None, None, *[None] * 8, *extra, None, None, C.byref(h))
    assert rc == pd.PDLP_ERR_INVALID_ARGUMENT and not h.value
    m = np.array([3, 2], np.int32)
    n = np.array([4, 0], np.int32)        # instance 1 has no columns
    nnz = np.array([5, 1], np.int64)
    rc = f(2, m.ctypes.data_as(pd.I32), n.ctypes.data_as(pd.I32),
           nnz.ctypes.data_as(C.POINTER(C.c_int64)), *[None] * 8, *extra, None, None, C.byref(h))
    assert rc == pd.PDLP_ERR_INVALID_ARGUMENT and not h.value
    assert "instance 1" in pd.lib().pdlp_last_error().decode()
    n[1] = 3
    rc = f(2, m.ctypes.data_as(pd.I32), n.ctypes.data_as(pd.I32),
           nnz.ctypes.data_as(C.POINTER(C.c_int64)), *[None] * 8, *extra, None, None, C.byref(h))
    assert rc == pd.PDLP_ERR_INVALID_ARGUMENT and not h.value
    assert "NULL" in pd.lib().pdlp_last_error().decode()


def test_from_tensors_checks_before_the_library():
    """Batch/Unroll.from_tensors refuse host tensors, wrong dtypes and wrong
    lengths in Python, before any call into the library."""
    torch = pytest.importorskip("torch")
    lp = _tiny()
    m, n, nnz = [len(lp["lc"])], [len(lp["c"])], [len(lp["col"])]
    ts = [torch.as_tensor(lp[k]) for k in ("row_ptr", "col", "val", "c", "lc", "uc", "lv", "uv")]
    for cls in (pd.Batch, pd.Unroll):
        with pytest.raises(ValueError, match="CUDA tensors"):
            cls.from_tensors(m, n, nnz, *ts)
        with pytest.raises(ValueError, match="n >= 1"):
            cls.from_tensors(m, [0], nnz, *ts)
        with pytest.raises(ValueError, match="one entry per instance"):
            cls.from_tensors(m + m, n, nnz, *ts)
