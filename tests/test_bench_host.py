"""Host logic of the benchmark: the one-GPU refusal, the roofline's work units and the gate on the
stored HBM traffic reference (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1608_05794_amd import synth  # noqa: E402


def _args(*argv):
    old = sys.argv
    sys.argv = ["bench.py", *argv]
    try:
        return bench.parse()
    finally:
        sys.argv = old


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "--gpus must be 1" in r.stderr and r.stdout == ""


def test_work_units_of_the_roofline():
    # per attempted ROS4 step: the Jacobian, two source terms, the iteration matrix, a dense LU of
    # (2/3) N^3 and four solves of 2 N^2 each (the counts the stored figures were computed with)
    w53 = bench.algorithmic_flops(bench.mech_structure(synth.mechanism_file("M53")))
    assert w53["ros4_step"] == 260413
    N = 54
    assert w53["lu"] == (2 * N ** 3) // 3
    assert w53["ros4_step"] == w53["jac"] + 2 * w53["rhs"] + N * N + w53["lu"] + 8 * N * N + 24 * N
    w111 = bench.algorithmic_flops(bench.mech_structure(synth.mechanism_file("M111")))
    assert 1.3e6 < w111["ros4_step"] < 1.45e6
    assert w111["rhs"] > w53["rhs"] > 0 and w111["jac"] > w111["rhs"]


def test_traffic_reference_applies_only_to_its_workload_and_sources(monkeypatch):
    ref = bench.measured_traffic(_args())
    # bytes per launch of the default command while the kernel sources match the counter runs
    assert ref is None or 1e9 < ref < 1e13
    assert bench.measured_traffic(_args("--reactors", "1024")) is None
    assert bench.measured_traffic(_args("--mech", "M111")) is None
    assert bench.measured_traffic(_args("--precision", "fp32_refine")) is None
    # a source hash that does not match: the stored counters no longer describe the kernel
    monkeypatch.setitem(bench.TRAFFIC_REF, "sha256", "0" * 64)
    assert bench.measured_traffic(_args()) is None
