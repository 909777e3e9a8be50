"""The bench line's host-side logic (CPU): the one-GPU refusal, the byte model
of the roofline, and the rule that counted HBM traffic and VALU counts are
reported only for the force kernel, evaluator, workload and sources they were
taken with."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    run = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert run.returncode == 2
    line = json.loads(run.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_force_pass_byte_model():
    # x and F' (32) + v read and written (48) + drifted x (24) + each unordered pair's index once
    assert bench.force_kernel_bytes_per_atom(0.0) == 104.0
    assert bench.force_kernel_bytes_per_atom(27.8) == pytest.approx(104.0 + 55.6)
    # the whole step: both passes plus the build spread over its period
    assert bench.step_bytes_per_atom(27.8, 10) == pytest.approx(136.0 + 4 * 27.8 + (56.0 + 2 * 27.8) / 10)


def _run(evaluator, kernel=1):
    return {"force_kernel_us": 90.0, "autotuned": {"kernel": kernel, "evaluator": evaluator}, "value": 5e9}


@pytest.mark.parametrize("prec,evaluator", [("fp64", 0), ("fp64", 1), ("mixed", 0)])
def test_counted_traffic_for_the_kernel_it_was_taken_on(prec, evaluator):
    r = bench.roofline_for(_run(evaluator), prec, 27.8, 1013760, 10, "bcc1m", None)
    t = bench.FORCE_TRAFFIC[(prec, evaluator)]
    if bench.force_sources_hash() != t["sources_sha256_16"]:
        pytest.skip("force kernel sources changed since the counters were taken")
    expect = 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])
    assert r["traffic_bytes_per_launch"] == expect
    assert r["traffic"] == pytest.approx(expect / 90e-6 / 1e9)
    assert r["alu"]["valu_instr_per_wave"] == t["valu_per_wave"]
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["achieved"] == pytest.approx(bench.force_kernel_bytes_per_atom(27.8) * 1013760 / 90e-6 / 1e9)


def test_no_traffic_for_other_kernels_workloads_or_sources(monkeypatch):
    assert bench.roofline_for(_run(1), "mixed", 27.8, 1013760, 10, "bcc1m", None)["traffic"] is None  # not counted
    assert bench.roofline_for(_run(0, kernel=0), "fp64", 27.8, 1013760, 10, "bcc1m", None)["traffic"] is None
    assert bench.roofline_for(_run(0), "fp64", 27.8, 1013760, 10, "fec256", None)["traffic"] is None
    monkeypatch.setattr(bench, "force_sources_hash", lambda: "0000000000000000")
    r = bench.roofline_for(_run(0), "fp64", 27.8, 1013760, 10, "bcc1m", None)
    assert r["traffic"] is None and r["alu"] is None and r["frac"] > 0
