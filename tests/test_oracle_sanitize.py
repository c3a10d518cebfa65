"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

tests/oracle_sanitize.c drives every oracle entry point on small 1-, 2- and
3-D inputs, both modes and several thread counts; built with gcc's
sanitizers (no recovery), any out-of-bounds access, leak or undefined
operation in oracle/oracle.c fails the run.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_runs_clean_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-o", exe,
           os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HERE, "oracle_sanitize.c"),
           "-lm", "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = ("detect_leaks=1:abort_on_error=0:halt_on_error=1:"
                           "verify_asan_link_order=0")
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle sanitizer run ok" in r.stdout
