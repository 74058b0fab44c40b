"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/native/build_sanitized.py builds a copy of libpdlp.so from the same
sources with only the host code instrumented (every sanitizer flag goes to
the host compilation through -Xarch_host; the GPU code is built as usual) and
links tests/native/pdlp_host_sanitize.cpp against it.  The driver calls every
entry point of the C ABI on small synthetic LPs: validation and rejections,
single problems with the default, two-phase, autotuned and eager schedules,
polishing, warm starts, state export and import, the normalized gap, the
allocation-free product, an infeasible problem, the Algorithm 5 mode,
batches (host and device input, graphs on and off) and the unrolled map
(forward, replay, backward, tangent and their device variants).  Any memory
or undefined-behaviour error in the host code aborts the run.

On the CPU only the calls that must fail before any GPU work run, with leak
detection on, and a negative control shows that the instrumentation is live:
a caller array one entry short is caught inside the library's validation.
"""
import glob
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
NATIVE = os.path.join(HERE, "native")
EXE = os.path.join(NATIVE, "_build", "pdlp_host_sanitize")


def _sources():
    return (glob.glob(os.path.join(ROOT, "paper_2501_07018_amd", "csrc", "*")) +
            [os.path.join(ROOT, "include", "pdlp.h"),
             os.path.join(NATIVE, "pdlp_host_sanitize.cpp")])


def _stale():
    if not os.path.exists(EXE):
        return True
    t = os.path.getmtime(EXE)
    return any(os.path.getmtime(f) > t for f in _sources())


def _build():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "build_sanitized", os.path.join(NATIVE, "build_sanitized.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.build()


def _run(mode, leaks, timeout):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = f"detect_leaks={int(leaks)}:protect_shadow_gap=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    return subprocess.run([EXE, mode], capture_output=True, text=True, timeout=timeout, env=env)


@pytest.fixture(scope="module")
def built_here():
    if _stale():
        _build()
    return EXE


def test_rejections_run_clean_under_asan_and_ubsan(built_here):
    r = _run("cpu", leaks=True, timeout=120)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "done, 0 failure(s)" in r.stdout


def test_the_instrumentation_catches_a_short_caller_array(built_here):
    r = _run("overflow", leaks=False, timeout=120)
    assert r.returncode != 0 and "not detected" not in r.stdout
    assert "heap-buffer-overflow" in r.stderr, r.stderr[-4000:]
    assert "pdlp::host::validate" in r.stderr, r.stderr[-4000:]


@pytest.mark.gpu
def test_every_entry_point_runs_clean_under_host_sanitizers():
    print("[test] host-sanitized driver, every entry point", flush=True)
    assert not _stale(), "the sanitized build is missing or older than its sources: run build()"
    r = _run("gpu", leaks=False, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "done, 0 failure(s)" in r.stdout, r.stdout[-2000:]
