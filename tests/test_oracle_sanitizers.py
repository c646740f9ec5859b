"""The oracle's C code (exactdot.c) under AddressSanitizer and
UndefinedBehaviorSanitizer: a host driver (tests/native/exactdot_driver.c)
runs every branch of the exact dot product -- subnormal, huge and cancelling
products, strided rows, empty rows, a row long enough for the accumulator's
periodic carry resolution -- and checks the certified fast path against the
superaccumulator bit for bit and sums with an integer closed form.  Any
memory error or undefined behaviour aborts the driver."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_exactdot_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc is not installed")
    exe = tmp_path / "exactdot_asan"
    cmd = [gcc, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-fopenmp", "-ffp-contract=off", os.path.join(ROOT, "oracle", "exactdot.c"),
           os.path.join(HERE, "native", "exactdot_driver.c"), "-o", str(exe), "-lm"]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and "asan" in build.stderr.lower():
        pytest.skip("the sanitizer runtimes are not installed: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0 and run.stdout.strip().endswith("ok"), run.stdout + run.stderr
