"""Host-side pieces of bench.py's reporting: the one-GPU refusal, the
roofline's per-launch work of the order-3 sampled pass, and the check that
ties the recorded HBM traffic to the kernel source it was measured on."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)   # defines functions only; main() runs under __main__
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_sampled_pass_work_per_launch_for_the_n400_order3_workload(bench):
    # per sample: prefix chain r1 r2 = 100 FMAs, suffix chain 100, middle-core
    # outer product 100, plus r1 + 2 r2 for the boundary cores: 330 FMAs
    shape, ranks, n = [400, 400, 400], [1, 10, 10, 1], 640_000
    assert bench.sampled_pass_flops(shape, ranks, n) == 2 * 330 * n == 422_400_000
    # three int32 indices and one value per sample
    assert bench.sampled_pass_bytes(shape, n, 8) == 20 * n
    assert bench.sampled_pass_bytes(shape, n, 4) == 16 * n


def test_sampled_pass_work_per_launch_for_the_order14_workload(bench):
    # ranks (1,4,8,...,8,4,1): S = 4*8 + 10*64 + 8*4 = 704; per sample
    # 3 S + r_1 + 2 r_13 = 2124 FMAs
    shape = [4] * 14
    ranks = [1, 4] + [8] * 11 + [4, 1]
    assert bench.sampled_pass_flops(shape, ranks, 2_000_000) == 2 * 2124 * 2_000_000
    assert bench.sampled_pass_bytes(shape, 2_000_000, 8) == (4 * 14 + 8) * 2_000_000


@pytest.mark.parametrize("workload", ["c2", "c4", "hbm3"])
def test_recorded_traffic_matches_the_current_kernel_source(bench, workload):
    path = bench.traffic_path(workload)
    if not os.path.exists(path):
        pytest.skip(f"no traffic record for {workload} yet")
    with open(path) as f:
        rec = json.load(f)
    if rec["source_sha256_16"] != bench.kernel_source_hash(workload):
        assert bench.measured_traffic("fp64", workload) is None
        return
    for prec in ("fp64", "mixed"):
        leg = rec[prec]
        assert bench.measured_traffic(prec, workload) == leg["bytes_per_launch"]
        # what the counters saw is of the order of the index/value stream: the
        # chain kernel reads the shared leading index rows once per chunk, so
        # it may read less than the full stream, never a small fraction of it
        assert leg["bytes_per_launch"] >= 0.5 * leg["algorithmic_bytes_per_launch"]


def test_recorded_traffic_is_dropped_once_the_kernel_changes(bench, monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda workload="c2": "0" * 16)
    assert bench.measured_traffic("fp64", "c2") is None
