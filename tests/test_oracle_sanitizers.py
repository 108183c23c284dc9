"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(CPU): tests/oracle_sanitize_main.c drives every oracle entry point over the
operator's edge cases on exactly sized heap buffers; any out-of-bounds access,
leak or undefined arithmetic aborts the run with a report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "tests", "oracle_sanitize_main.c"),
           os.path.join(ROOT, "oracle", "msda_oracle.c"), "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ)
    # halt on the first report; leak checking on; do not insist on being
    # first in the library list
    env["ASAN_OPTIONS"] = "halt_on_error=1:detect_leaks=1:verify_asan_link_order=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "4"
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    assert res.stdout.strip().endswith("ok"), res.stdout[-2000:]
    assert "runtime error" not in res.stderr, res.stderr[-4000:]
