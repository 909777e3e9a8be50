"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): tests/sanitize_abi.cpp drives md_create's validation, the table
construction, workspace planning and the option switches through the C ABI,
linked against an instrumented build of md_runtime.hip (the host half; the
device half and the kernel launchers come from libmdeam.so, which this run
never reaches)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1107_2619_amd")
HIPCC = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")


def test_host_library_under_sanitizers(tmp_path):
    if not os.path.exists(HIPCC) or not os.path.exists(os.path.join(PKG, "libmdeam.so")):
        pytest.skip("hipcc or the built library is missing")
    exe = str(tmp_path / "sanitize_abi")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", f"-I{ROOT}",
           os.path.join(ROOT, "tests", "sanitize_abi.cpp"), os.path.join(PKG, "csrc", "md_runtime.hip"),
           f"-L{PKG}", "-lmdeam", f"-Wl,-rpath,{PKG}", "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert build.returncode == 0, build.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env, cwd=str(tmp_path))
    out = run.stdout + run.stderr
    assert run.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert " 0 failures" in run.stdout
    shutil.rmtree(tmp_path, ignore_errors=True)
