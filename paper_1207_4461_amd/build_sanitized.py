"""Host-sanitizer build of libqbx for CPU runs of the host checks.

build_sanitized() compiles every source with AddressSanitizer and
UndefinedBehaviorSanitizer on the host side only (each flag after -Xarch_host,
so the GPU code is the ordinary one) into _build_san/libqbx_san.so.  A child
process loads it with sanitizer_env(): the clang sanitizer runtime preloaded
and QBX_LIB pointing at the library, e.g.

    python -m paper_1207_4461_amd.build_sanitized
    env $(...) python -m pytest tests/test_boundary.py     # see sanitizer_env()
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

from paper_1207_4461_amd.build import COMMON, CSRC, HERE, SOURCES, _compile, _entry, _hipcc

BUILD_SAN = os.path.join(HERE, "_build_san")
LIB_SAN = os.path.join(BUILD_SAN, "libqbx_san.so")
SAN_FLAGS = ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host",
             "-fno-omit-frame-pointer"]


def _san_runtime() -> str:
    """The clang AddressSanitizer runtime of the ROCm toolchain (shared build)."""
    root = "/opt/rocm/llvm/lib/clang"
    for ver in sorted(os.listdir(root), reverse=True) if os.path.isdir(root) else []:
        cand = os.path.join(root, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(cand):
            return cand
    raise RuntimeError("libclang_rt.asan-x86_64.so not found under " + root)


def build_sanitized(verbose: bool = False, force: bool = False) -> str:
    """Compile every source with the host sanitizers into _build_san and link
    libqbx_san.so there (the sanitizer runtime is resolved at load time)."""
    os.makedirs(BUILD_SAN, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, _entry(s)[0]))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, force, BUILD_SAN, SAN_FLAGS), srcs))
    tmp = LIB_SAN + ".tmp"
    cmd = [_hipcc(), *COMMON, "-shared", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB_SAN)
    return LIB_SAN


def sanitizer_env() -> dict:
    """Environment for a child process that loads libqbx_san.so: the runtime
    preloaded, leak checks off (the interpreter's own allocations are not ours)."""
    env = dict(os.environ)
    env["LD_PRELOAD"] = _san_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["QBX_LIB"] = LIB_SAN
    return env


if __name__ == "__main__":
    print(build_sanitized(verbose="-v" in sys.argv))
