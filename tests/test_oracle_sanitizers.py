"""The oracle built with gcc's AddressSanitizer and UndefinedBehaviorSanitizer
(a separate program, oracle/sanitize_check.c, that drives every public routine
on tiny two- and three-level problems): no memory error, no undefined
behaviour, and the solves still reach their residual."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_and_ubsan():
    src = os.path.join(ROOT, "oracle", "sanitize_check.c")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "sanitize_check")
        cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-o", exe, src, "-lm"]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="abort_on_error=0:halt_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "sanitize_check ok" in r.stdout
