"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) and run through every exported function on small mixed-q
models by ``oracle_sanitize_driver.c``: no sanitizer report, exit status 0."""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile

import pytest

from oracle import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "orc_asan")
        subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                               "-o", exe, oracle.SRC, os.path.join(HERE, "oracle_sanitize_driver.c"),
                               "-lm"])
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, r.stderr[-4000:]
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
        assert "sanitized oracle run ok" in r.stdout
