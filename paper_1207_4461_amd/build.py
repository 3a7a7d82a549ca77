"""Build libqbx.so (HIP, gfx950) in-tree with hipcc.

Every source under csrc/ is compiled as HIP for gfx950, one object per
source (in parallel), then linked into paper_1207_4461_amd/libqbx.so.
(build_sanitized.py builds a host-sanitizer copy for CPU runs of the host checks.)
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libqbx.so")

# (source, object name, extra flags), slowest first; the batched forward source is
# compiled once per mode
SOURCES = [("qbx_batched_fwd.hip", "qbx_batched_fwd1", ["-DQBX_FWD_MODE=1"]),
           ("qbx_batched_fwd.hip", "qbx_batched_fwd0", ["-DQBX_FWD_MODE=0"]),
           "qbx_batched_adj.hip", "qbx_batched_fused.hip",
           "qbx_adjoint.hip", "qbx_forward.hip", "qbx_explicit.hip", "qbx_batched.hip",
           "qbx_geometry.hip", "qbx_split.hip", "qbx_solve.hip", "qbx_noalloc.hip",
           "qbx_expansions.hip",
           "qbx_api.cpp", "qbx_autotune.cpp"]
ARCH = os.environ.get("QBX_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def _up_to_date(src: str, obj: str) -> bool:
    if not os.path.exists(obj):
        return False
    t = os.path.getmtime(obj)
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, h) for h in os.listdir(CSRC)
                                        if h.endswith(".h")]
    deps.append(os.path.join(os.path.dirname(HERE), "include", "qbx.h"))
    return all(os.path.getmtime(d) < t for d in deps)


def _entry(e):
    """(source, object name, extra flags) of a SOURCES entry."""
    if isinstance(e, str):
        return e, os.path.splitext(e)[0], []
    return e


def _compile(entry, verbose: bool, force: bool = True, outdir: str = BUILD,
             extra=()) -> str:
    src, name, flags = _entry(entry)
    flags = [*flags, *extra]
    obj = os.path.join(outdir, name + ".o")
    if not force and _up_to_date(src, obj):
        return obj
    cmd = [_hipcc(), "-x", "hip", *COMMON, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = False, force: bool = True) -> str:
    """Compile every source (force=False: only those older than their inputs) and link."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, _entry(s)[0]))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, force), srcs))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), *COMMON, "-shared", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, force="--incremental" not in sys.argv))
