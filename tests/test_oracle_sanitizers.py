"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

oracle/sanitize_driver.c is compiled with the oracle's sources and
-fsanitize=address,undefined (no recovery) and run on LPs that reach every
path of the solver: a planted LP (with and without polishing), a planted
primal-infeasible LP, a tiny LP with free and ranged rows and infinite
bounds, an LP with an empty row and column, and an LP without rows; each
also runs the unrolled map's replay, adjoint and tangent.  Any memory or
undefined-behaviour error aborts the run."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import lpgen

HERE = os.path.dirname(os.path.abspath(__file__))
ORC = os.path.join(os.path.dirname(HERE), "oracle")


def _write(lp, path):
    with open(path, "wb") as f:
        np.array([lp.m, lp.n], dtype=np.int32).tofile(f)
        np.array([int(np.asarray(lp.row_ptr)[-1])], dtype=np.int64).tofile(f)
        np.asarray(lp.row_ptr, dtype=np.int32).tofile(f)
        np.asarray(lp.col, dtype=np.int32).tofile(f)
        for k in ("val", "c", "lc", "uc", "lv", "uv"):
            np.asarray(getattr(lp, k), dtype=np.float64).tofile(f)


def _lps():
    import scipy.sparse as sp
    out = [lpgen.planted_uniform(80, 150, 5, seed=7), lpgen.tiny_random_lp(3, 6, 9)]
    out.append(lpgen.infeasible_lp("primal", 0, 60, 90))
    out.append(lpgen.infeasible_lp("dual", 0, 60, 90))
    rng = np.random.default_rng(2)
    dense = np.round(rng.standard_normal((12, 20)) * (rng.random((12, 20)) < 0.3), 2)
    dense[4] = 0.0
    dense[:, 7] = 0.0
    A = sp.csr_matrix(dense)
    A.sort_indices()
    x0 = rng.uniform(0, 1, 20)
    b = dense @ x0
    out.append(lpgen.LP(12, 20, A.indptr.astype(np.int32), A.indices.astype(np.int32),
                        A.data, rng.standard_normal(20), b - 0.5, b + 0.5, np.zeros(20),
                        np.ones(20)))
    out.append(lpgen.LP(0, 4, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0),
                        np.array([1.0, -1.0, 0.0, 2.0]), np.zeros(0), np.zeros(0),
                        -np.ones(4), np.ones(4)))
    return out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "orc_san"
    srcs = [os.path.join(ORC, f) for f in ("sanitize_driver.c", "pdlp_oracle.c",
                                           "pdlp_oracle_unroll.c")]
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-Wno-unknown-pragmas",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I" + ORC, *srcs, "-o", str(exe), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr + r.stdout).lower():
        pytest.skip("the sanitizer runtime is not installed: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    for i, lp in enumerate(_lps()):
        path = tmp_path / f"lp{i}.bin"
        _write(lp, path)
        run = subprocess.run([str(exe), str(path)], capture_output=True, text=True, env=env,
                             timeout=300)
        assert run.returncode == 0, (i, run.stdout[-500:], run.stderr[-3000:])
        assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr, \
            run.stderr[-3000:]
        assert "unroll K=40" in run.stdout
