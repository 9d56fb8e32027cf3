"""The oracle's pins, run on a build of the oracle with AddressSanitizer
and UndefinedBehaviorSanitizer (CPU only).

An out-of-bounds access, a use after free or undefined behaviour anywhere
the pins reach in oracle.c aborts the child run, and the test fails.  The
ASan runtime is preloaded into a child interpreter, which loads the
sanitized library through ORACLE_LIB.  Leak checking is off: the
interpreter itself holds memory at exit.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    if not shutil.which("gcc"):
        return None
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    try:
        import build as oracle_build
    finally:
        sys.path.pop(0)
    lib = oracle_build.build_sanitized(str(tmp_path / "liboracle_sanitized.so"))
    env = dict(os.environ, LD_PRELOAD=asan, ORACLE_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    tests = [os.path.join(ROOT, "tests", f) for f in
             ("test_oracle_pins.py", "test_oracle_sw_three_body.py", "test_oracle_multi.py",
              "test_oracle_green_kubo.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", *tests], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
