"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host
code, gcc) runs two capillaries with walls, forcing and an invalid input
without a memory or undefined-behaviour error."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_asan"
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "oracle"), os.path.join(ROOT, "oracle", "lb_oracle.c"),
           os.path.join(ROOT, "tests", "oracle_sanitize_main.c"), "-o", str(exe), "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "model 1 ok" in r.stdout and "model 0 ok" in r.stdout
