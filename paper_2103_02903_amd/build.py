"""Build step of the HIP library ``libmrlbm.so`` for gfx950 (in-tree)."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libmrlbm.so")
SOURCES = [os.path.join(PKG, "csrc", "mrlbm.hip")]
DEPS = SOURCES + [os.path.join(PKG, "csrc", f) for f in ("mr_device.h", "mr_kernels.h", "mr_kernels3d.h", "mr_adjoint.h")] + [
    os.path.join(ROOT, "include", "mrlbm.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # the mesh decisions compare details computed in a prescribed operation order
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile ``csrc/*.hip`` into ``libmrlbm.so`` next to this file."""
    if not force and os.path.exists(LIB) and all(os.path.getmtime(LIB) >= os.path.getmtime(d) for d in DEPS):
        return LIB
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, *SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
