"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(g++, host code only) and driven by tests/sanitize/oracle_driver.cpp: seeded
tables of every encoding, queries with every predicate kind, OR clauses,
keys, SUM / MIN / MAX and two-column expressions, answers checked against
the driver's own row-by-row evaluation.  Any sanitizer report fails."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_asan_and_ubsan(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path / "oracle_asan")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           os.path.join(ROOT, "oracle", "ccq_oracle.cpp"),
                           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.cpp"), "-o", exe, "-lpthread"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "queries checked" in r.stdout
