"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) runs every entry point on edge shapes (1x1, 1xN, Nx1,
radius beyond the image, volumes) with no sanitizer report."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_oracle")
    srcs = [os.path.join(HERE, "sanitize_oracle.c")] + [
        os.path.join(ORACLE, f) for f in ("osbf_oracle.c", "osbf3d_oracle.c", "osbf_gauss_oracle.c")]
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-o", exe, *srcs, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr
    assert "sanitize_oracle: ok" in res.stdout
