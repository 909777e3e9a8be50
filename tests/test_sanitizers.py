"""Host sanitizers on the oracle (CPU): the oracle's C source and a driver
that runs every entry point on small periodic systems (orthorhombic and
sheared cells, every integrator), built with AddressSanitizer and
UndefinedBehaviorSanitizer, with and without OpenMP threads."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("openmp", [False, True])
def test_oracle_under_asan_and_ubsan(tmp_path, openmp):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = tmp_path / "sanitize_oracle"
    cmd = ["gcc", "-std=c11", "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-Wall", "-Wno-unknown-pragmas", "-o", str(exe),
           os.path.join(HERE, "sanitize_oracle.c"), "-lm"]
    if openmp:
        cmd.insert(1, "-fopenmp")
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, OMP_NUM_THREADS="4", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "runtime error" not in run.stderr and "ERROR: AddressSanitizer" not in run.stderr
    assert run.stdout.startswith("rc 0 checksum")
