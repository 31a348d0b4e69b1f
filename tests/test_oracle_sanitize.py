"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer:
gcc builds oracle/oracle.c and cpu_baseline/ruling_set.c with a small C driver
(host code only) and runs it on valid and malformed lists (plain, weighted,
and the multi-threaded CPU baseline), graphs and both batched forms."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "oracle_sanitized"
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-pthread",
           os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "cpu_baseline", "ruling_set.c"),
           os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr and "not supported" in r.stderr:
        pytest.skip("sanitizers not supported by this gcc")
    assert r.returncode == 0, r.stderr
    # verify_asan_link_order=0: the environment may preload other libraries
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert run.returncode == 0 and run.stdout.strip() == "OK", run.stdout + run.stderr
