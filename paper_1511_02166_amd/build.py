"""Build the gfx950 HIP library ``libpanel.so`` in-tree with hipcc.

Run ``python -m paper_1511_02166_amd.build`` (or call ``build()``).  Every
source is compiled to its own object (in parallel), then the objects are
linked into the shared object next to this file, which is what the Python
binding, the tests and the benchmark load.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "libpanel.so")
ARCH = os.environ.get("PANEL_OFFLOAD_ARCH", "gfx950")

SOURCES = ["panel_abi.cpp", "geometry.hip", "assemble.hip", "assemble_hs.hip", "lu.hip", "lu_wave.hip", "forces.hip",
           "adjoint.hip", "adjoint_wave.hip", "viscous.hip", "ga.hip", "mathcheck.hip"]

FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # keep the compiler from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the HIP library)")


def _filter(stderr: str) -> str:
    # the host pass does not know the packed-FP32 feature flag: harmless
    return "\n".join(l for l in (stderr or "").splitlines() if "packed-fp32-ops" not in l)


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    errs = _filter(res.stderr)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}): {' '.join(cmd)}\n{errs}")
    if verbose and errs.strip():
        print(errs, file=sys.stderr)


def _stale(src: str, obj: str) -> bool:
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith((".hpp", ".h"))]
    deps.append(os.path.join(os.path.dirname(HERE), "include", "panel.h"))
    return any(os.path.getmtime(d) > t for d in deps if os.path.exists(d))


def build(verbose: bool = False, jobs: int | None = None, force: bool = True) -> str:
    """Compile every source (``force=False``: only objects older than their
    source or any header) and link ``libpanel.so``."""
    os.makedirs(OBJ, exist_ok=True)
    cc = hipcc()
    objs = []
    cmds = []
    for s in SOURCES:
        o = os.path.join(OBJ, os.path.splitext(s)[0] + ".o")
        objs.append(o)
        src = os.path.join(CSRC, s)
        if force or _stale(src, o):
            cmds.append([cc] + FLAGS + ["-x", "hip", "-c", src, "-o", o])
    jobs = jobs or max(1, min(len(cmds), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = LIB + ".tmp"
    _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC"] + objs + ["-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, force="--changed" not in sys.argv))
