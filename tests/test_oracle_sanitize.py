"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer: every
entry point of oracle/oracle.c runs once on small inputs in an executable built
with both sanitizers (tests/asan/oracle_asan.c), which must exit cleanly with
no report (leaks included)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    src = [os.path.join(ROOT, "tests", "asan", "oracle_asan.c"),
           os.path.join(ROOT, "oracle", "oracle.c")]
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fno-fast-math", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-pthread", *src, "-o", exe, "-lm"])
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1:verify_asan_link_order=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle sanitizer run: ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
