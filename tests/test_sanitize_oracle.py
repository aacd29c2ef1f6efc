"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle's C source is built once more with every out-of-bounds access,
use after free, signed overflow, bad shift and misaligned or null access made
fatal (oracle/build.py, SAN_FLAGS), and the oracle pin tests run against that
build in a child process with the sanitizer runtimes preloaded.  The pins
exercise every oracle routine the GPU path is checked against: MST builders
(exact and divide-and-conquer), tree transforms, forces and their tangents,
leapfrog, GBS steps and the driver, rebuilds, replays and round trips.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    sys.path.insert(0, ROOT)
    from oracle import build as ob
    lib = ob.build_sanitized(str(tmp_path / "liborc_san.so"))
    env = dict(os.environ)
    env.update({
        "MSTAR_ORACLE_LIB": lib,
        "LD_PRELOAD": f"{asan}:{ubsan}",
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",   # the interpreter's own leaks are not the oracle's
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "OMP_NUM_THREADS": "4",
    })
    files = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu and not slow", "-p",
                        "no:cacheprovider", *files], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=1500)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out, out[-2000:]
