"""Build libpppm_mi355x.so: the HIP kernels and the C ABI, for gfx950 only.

    python -m paper_1702_04250_amd.build

compiles every ``csrc/*.hip`` with hipcc into ``paper_1702_04250_amd/lib/``
(in-tree, so the built library travels with the source tree).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
INCLUDE = ROOT / "include"
LIBDIR = PKG / "lib"
LIBNAME = "libpppm_mi355x.so"

ARCH = "gfx950"
# -packed-fp32-ops: keep the compiler from emitting packed FP32 VALU ops.
HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the MI355X library cannot be built")
    return path


def build(verbose: bool = False) -> Path:
    """Compile the library (always recompiles) and return its path."""
    LIBDIR.mkdir(exist_ok=True)
    sources = sorted(str(p) for p in CSRC.glob("*.hip"))
    out = LIBDIR / LIBNAME
    tmp = LIBDIR / (LIBNAME + ".tmp")
    cmd = [hipcc(), *HIP_FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", *sources,
           "-L/opt/rocm/lib", "-lrocfft", "-Wl,-rpath,/opt/rocm/lib", "-o", str(tmp)]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed ({res.returncode})")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    p = build(verbose=True)
    print(p)
