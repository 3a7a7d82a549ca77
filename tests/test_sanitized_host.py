"""The host checks (test_boundary.py) against the host-sanitizer build of the library
(AddressSanitizer and UndefinedBehaviorSanitizer on the host code; built by
``python -m paper_1207_4461_amd.build_sanitized``, about two minutes, so it is
skipped until that library exists).  The child process must really have loaded
that library and the sanitizer runtime."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def BS():
    return pytest.importorskip("paper_1207_4461_amd.build_sanitized")


@pytest.fixture(scope="module")
def env(BS):
    if not os.path.exists(BS.LIB_SAN):
        pytest.skip("host-sanitizer library not built (python -m paper_1207_4461_amd.build_sanitized)")
    return BS.sanitizer_env()


def test_child_loads_the_sanitized_library(BS, env):
    code = ("from paper_1207_4461_amd import _lib; lib = _lib.load(); "
            "maps = open('/proc/self/maps').read(); "
            "print(_lib.LIB_PATH); print('asan' if 'libclang_rt.asan' in maps else 'no-asan'); "
            "print('san-lib' if 'libqbx_san.so' in maps else 'no-san-lib')")
    out = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True,
                         text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    lines = out.stdout.split()
    assert lines[0] == BS.LIB_SAN and "asan" in lines and "san-lib" in lines


def test_boundary_checks_pass_under_the_sanitizers(env):
    out = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                          os.path.join(HERE, "test_boundary.py")], env=env, cwd=ROOT,
                         capture_output=True, text=True, timeout=600)
    tail = "\n".join((out.stdout + out.stderr).splitlines()[-15:])
    assert out.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in out.stderr and "runtime error:" not in out.stderr
