"""Build libpppm_mi355x.so: the HIP kernels and the C ABI, for gfx950 only.

    python -m paper_1702_04250_amd.build

compiles every ``csrc/*.hip`` with hipcc and every ``csrc/*.cpp`` (host-only
C++) with g++ into ``paper_1702_04250_amd/lib/`` (in-tree, so the built
library travels with the source tree).
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
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


HOST_CXX = "g++"
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall"]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the MI355X library cannot be built")
    return path


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed ({res.returncode}): {cmd[-1]}")


def build(verbose: bool = False) -> Path:
    """Compile the library (always recompiles) and return its path.  The
    sources compile in parallel (one hipcc per file), then link."""
    from concurrent.futures import ThreadPoolExecutor

    LIBDIR.mkdir(exist_ok=True)
    objdir = LIBDIR / "obj"
    objdir.mkdir(exist_ok=True)
    sources = sorted(CSRC.glob("*.hip"))
    host_sources = sorted(CSRC.glob("*.cpp"))  # plain host C++ (parameter logic)
    objs = [objdir / (p.stem + ".o") for p in sources + host_sources]
    cmds = [[hipcc(), *HIP_FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", "-c", str(src), "-o", str(obj)]
            for src, obj in zip(sources, objs)]
    cmds += [[HOST_CXX, *HOST_FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", "-c", str(src), "-o", str(objdir / (src.stem + ".o"))]
             for src in host_sources]
    workers = max(1, min(len(cmds), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    out = LIBDIR / LIBNAME
    tmp = LIBDIR / (LIBNAME + ".tmp")
    _run([hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *map(str, objs),
          "-L/opt/rocm/lib", "-lrocfft", "-Wl,-rpath,/opt/rocm/lib", "-o", str(tmp)], verbose)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    p = build(verbose=True)
    print(p)
