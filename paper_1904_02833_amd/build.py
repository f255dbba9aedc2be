"""Build the gfx950 HIP library ``libsnake.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libsnake.so")
SOURCES = ["step.hip", "newton.hip", "gs.hip", "carriage.hip", "index.hip", "api.hip", "mlp.hip", "link.hip"]
# host-sanitized variant for CPU checks of the host paths (descriptor
# validation, workspace sizing, tile planning); its flags are the caller's
SAN_LIB = os.path.join(HERE, "libsnake_san.so")

# Packed FP32 instructions are kept out of the generated code; contraction
# follows source expressions only, so one device function compiles to the
# same arithmetic in every kernel that inlines it.
HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    "-ffp-contract=on",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False, out: str = LIB, extra_flags=()) -> str:
    """Compile every source into ``out``; ``extra_flags`` follow the standard
    ones (a later -O wins)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, *extra_flags, "-I", INCLUDE, "-I", CSRC, "-o", tmp,
           *[os.path.join(CSRC, s) for s in SOURCES]]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stderr)
    if verbose:
        print(" ".join(cmd))
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
