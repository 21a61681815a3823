"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

A small C driver (tests/sanitize/oracle_driver.c) links the oracle sources,
builds and walks trees of small adversarial sets on both key curves, checks the
leaf-first reference against the top-down oracle and the Hilbert round trip;
any out-of-bounds access, leak or undefined operation aborts the run.
"""
import os
import shutil
import subprocess

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    srcs = [os.path.join(HERE, "sanitize", "oracle_driver.c"), oracle.SRC, oracle.LEAF_FIRST_SRC,
            oracle.GRAVITY_SRC]
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-o", exe, *srcs,
           "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "SANITIZED RUN OK" in r.stdout
