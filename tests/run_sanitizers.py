"""Run the CPU test suite under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds the oracle (clang, -O2) and the host side of the HIP library (hipcc,
-O1, sanitizers on the host code only: the device code is compiled as usual
and never runs here) with both sanitizers and the shared sanitizer runtime,
then runs ``pytest -m "not gpu"`` (or the given pytest arguments) in a child
process that preloads that runtime.  Leak detection is off: the Python
interpreter keeps its own allocations until exit.  Any sanitizer report
aborts the child and fails the run.  CPU only; no GPU is touched.

    python tests/run_sanitizers.py [pytest arguments]
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def runtime() -> str:
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        raise SystemExit("clang's shared AddressSanitizer runtime is not installed")
    return found[-1]


CLANG = "/opt/rocm/llvm/bin/clang"
# both sanitizers, shared runtime, the first report ends the process
ORACLE_CC = [CLANG, "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-shared-libsan", "-g"]
# hipcc: sanitize the host code only; -O1 keeps the build short (the device
# code never runs here)
HOST_FLAGS = ["-O1", "-g"] + [f for opt in ("-fsanitize=address", "-fsanitize=undefined",
                                            "-fno-sanitize-recover=undefined", "-shared-libsan",
                                            "-fno-omit-frame-pointer") for f in ("-Xarch_host", opt)]


def build() -> None:
    sys.path.insert(0, ROOT)
    os.environ["SNAKE_SANITIZE"] = "1"
    import oracle
    from paper_1904_02833_amd import build as hip_build

    print("[sanitize] oracle:", oracle.build(force=True, cc=ORACLE_CC), flush=True)
    print("[sanitize] library:", hip_build.build(out=hip_build.SAN_LIB, extra_flags=HOST_FLAGS), flush=True)


PLANTED = r"""
#include <stdlib.h>
int planted(int n) { int* a = malloc(n * sizeof(int)); a[n] = 1; int r = a[0]; free(a); return r; }
"""

CHECK = r"""
import ctypes, sys
sys.path.insert(0, %r)
import oracle, paper_1904_02833_amd as snk
assert oracle.LIB.endswith("liboracle_san.so") and snk.LIB_PATH.endswith("libsnake_san.so")
oracle.lib(); snk.lib()
ctypes.CDLL(None).__asan_init   # the preloaded runtime is live
ctypes.CDLL(%r).planted(4)      # must not return
"""


def self_check(env, tmp) -> None:
    """The sanitized libraries are the ones loaded, and a heap overflow in
    code built with the same flags is caught."""
    src, so = os.path.join(tmp, "planted.c"), os.path.join(tmp, "libplanted.so")
    open(src, "w").write(PLANTED)
    subprocess.check_call([*ORACLE_CC, "-O2", "-fPIC", "-shared", "-o", so, src])
    res = subprocess.run([sys.executable, "-c", CHECK % (ROOT, so)], env=env, capture_output=True, text=True)
    if res.returncode == 0 or "heap-buffer-overflow" not in res.stderr:
        raise SystemExit("sanitizer self-check failed:\n" + res.stderr[-2000:])
    print("[sanitize] self-check: sanitized libraries loaded, planted overflow caught", flush=True)


def main(argv) -> int:
    import tempfile

    build()
    env = dict(os.environ, SNAKE_SANITIZE="1", LD_PRELOAD=runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    with tempfile.TemporaryDirectory() as tmp:
        self_check(env, tmp)
    args = argv or ["tests", "-m", "not gpu", "-q", "-x", "-p", "no:cacheprovider"]
    return subprocess.call([sys.executable, "-m", "pytest", *args], cwd=ROOT, env=env)


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
