"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer:
the oracle is built with both (every finding fatal) and its pins for the
tree, lists, grid, columns, rates, upstream chain, H2 channel and kernel-
weighted luminosities run against that build in a child process.  A memory
error or undefined behaviour anywhere on those paths fails this test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_upstream.py", "tests/test_oracle_lw.py",
        "tests/test_oracle_kernel_lum.py"]


def _runtime(name):
    try:
        p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True, check=True)
    except (OSError, subprocess.CalledProcessError):
        return None
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_asan_and_ubsan():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    subprocess.run(["sh", os.path.join(ROOT, "oracle", "build.sh"), "sanitize"], check=True)
    env = dict(os.environ, ORACLE_LIB="liboracle_san.so", LD_PRELOAD=f"{asan} {ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "failed" not in r.stdout, tail
