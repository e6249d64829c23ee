"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds oracle/picard_oracle.c with its sanitizer driver (gcc, host code only) and runs
it: every exported oracle function is called on small random instances of both
policies, with and without node capacity, and must finish without a sanitizer report
(out-of-bounds access, leak, undefined behaviour) or a failed cross-check.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_sanitize")
        cmd = ["gcc", "-O1", "-g", "-std=c99", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-static-libasan",
               os.path.join(ROOT, "oracle", "picard_oracle.c"),
               os.path.join(ROOT, "oracle", "sanitize_driver.c"), "-o", exe, "-lm"]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, r.stderr[-4000:]
        assert "all oracle calls clean" in r.stdout
