"""Build of libzpl.so (gfx950) with hipcc, in the package directory."""
from __future__ import annotations

import os
import shutil
import subprocess
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
LIB = PKG / "libzpl.so"
SOURCES = ["zpl_kernels.hip", "zpl_api.cpp"]
ARCH = os.environ.get("ZPL_OFFLOAD_ARCH", "gfx950")

# -ffp-contract=off: every fused multiply-add in the device math is an explicit
# fma(), so results do not depend on where a function is inlined.
# -packed-fp32-ops: no packed FP32 instructions are generated.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
         "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall"]


def hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not Path(h).exists():
        raise RuntimeError("hipcc not found: ROCm is required to build libzpl")
    return h


def build(verbose: bool = False) -> Path:
    """Compile every HIP/C++ source of the library into libzpl.so."""
    tmp = LIB.with_suffix(".so.tmp%d" % os.getpid())
    cmd = [hipcc(), *FLAGS, *[str(CSRC / s) for s in SOURCES], "-o", str(tmp)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("libzpl build failed:\n" + r.stdout + r.stderr)
    if verbose:
        print(r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
