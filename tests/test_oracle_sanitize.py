"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer, on the
CPU: tests/oracle_sanitize_driver.c drives every call of its C interface on
small 2D and 3D cases (periodic, walls, open top, block, filter and BGK,
D3Q27 and D3Q19), and any out-of-bounds access, use after free, leak or
undefined operation ends the run with a sanitizer report and a non-zero
status."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    src = [os.path.join(HERE, "oracle_sanitize_driver.c"), os.path.join(ROOT, "oracle", "pulbm_oracle.c")]
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fopenmp", "-I", os.path.join(ROOT, "oracle"), "-o", exe, *src, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "oracle sanitizer run: ok" in r.stdout
