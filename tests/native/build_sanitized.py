"""Build the host-sanitized library and its driver (test infrastructure).

``libpdlp_san.so`` is libpdlp.so compiled from the same sources with the
host code instrumented by AddressSanitizer and UndefinedBehaviorSanitizer
(every sanitizer flag is passed to the host compilation only, through
-Xarch_host; the GPU code is built as usual).  ``pdlp_host_sanitize`` is the
driver of tests/native/pdlp_host_sanitize.cpp linked with the sanitizer
runtimes, which the instrumented library resolves against.  Both land in
tests/native/_build/.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(OUT, "libpdlp_san.so")
EXE = os.path.join(OUT, "pdlp_host_sanitize")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def build(verbose: bool = False):
    sys.path.insert(0, ROOT)
    from paper_2501_07018_amd import build as libbuild
    os.makedirs(OUT, exist_ok=True)
    flags = [f for f in libbuild.FLAGS if f != "-O3"] + ["-O1", "-g"]
    cmds = [
        [os.path.join(ROCM, "bin", "hipcc"), *flags, *HOST_SAN, "-Wl,-soname,libpdlp_san.so",
         "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(libbuild.HERE, "csrc"),
         *libbuild.SOURCES, "-o", LIB],
        [os.path.join(ROCM, "lib", "llvm", "bin", "clang++"), "-std=c++17", "-O1", "-g",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
         "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"),
         "-I" + os.path.join(ROOT, "include"), os.path.join(HERE, "pdlp_host_sanitize.cpp"),
         "-L" + OUT, "-lpdlp_san", "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
         "-Wl,-rpath,$ORIGIN", "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", EXE],
    ]
    for path in (LIB, EXE):
        if os.path.exists(path):
            os.remove(path)
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("sanitized build failed:\n" + r.stdout + r.stderr)
    return LIB, EXE


if __name__ == "__main__":
    print(build(verbose=True))
