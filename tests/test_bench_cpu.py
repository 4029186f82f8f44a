"""Host logic of bench.py, on the CPU: the algorithmic-byte unit the roofline
figure is built on, the stored counter readings it scales, and the refusal of
several GPUs."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes_per_frame():
    # depth 4 B per pixel, one 16-byte entry read per touched block, entry and
    # key written per new block (16 + 8), fp32 sum and weight read and written
    # per touched voxel (16)
    assert bench.algorithmic_bytes(307200, 0, 0, 0) == 4 * 307200
    assert bench.algorithmic_bytes(1, 10, 0, 0) == 4 + 160
    assert bench.algorithmic_bytes(1, 0, 10, 0) == 4 + 240
    assert bench.algorithmic_bytes(1, 0, 0, 10) == 4 + 160
    assert bench.algorithmic_bytes(640 * 480, 34308, 852, 1929532) == \
        4 * 640 * 480 + 16 * 34308 + 24 * 852 + 16 * 1929532
    # colour frames: the colour image, and the read and write of three
    # channel sums per touched voxel
    assert bench.algorithmic_bytes(100, 2, 1, 7, 3) == \
        bench.algorithmic_bytes(100, 2, 1, 7) + 4 * 100 + 8 * 3 * 7


def test_kernel_hash_is_stable():
    a, b = bench.kernel_sha(), bench.kernel_sha()
    assert a == b and len(a) == 16 and int(a, 16) >= 0


@pytest.mark.parametrize("name", [bench.TRAFFIC_FILE, bench.MULTI_TRAFFIC_FILE])
def test_stored_counter_readings_are_consistent(name):
    t = json.load(open(name))
    for k in ("kernel", "kernel_sha", "fetch_kib_per_dispatch", "write_kib_per_dispatch",
              "copy_calibration", "fetch_factor", "write_factor", "bytes_per_launch"):
        assert k in t, k
    cal = t["copy_calibration"]
    # the factors come from the calibration copy: it moves `bytes` each way
    assert t["fetch_factor"] == pytest.approx(cal["bytes"] / 1024 / cal["fetch_kib"], rel=1e-3)
    assert t["write_factor"] == pytest.approx(cal["bytes"] / 1024 / cal["write_kib"], rel=1e-3)
    want = (t["fetch_kib_per_dispatch"] * t["fetch_factor"]
            + t["write_kib_per_dispatch"] * t["write_factor"]) * 1024
    assert t["bytes_per_launch"] == pytest.approx(want, rel=1e-6)


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_host_report_names_the_cpu():
    h = bench.host_info()
    assert h["nproc"] == os.cpu_count() and 1 <= h["usable_cpus"] <= h["nproc"]
    assert h["cpu_model"] is None or isinstance(h["cpu_model"], str)
    assert 1 <= bench.cpu_threads() <= 16


def test_medians_over_passes():
    assert bench.med([3.0, 1.0, 2.0]) == 2.0
    assert bench.med([5.0]) == 5.0


def test_a_gpu_held_by_another_process_is_refused(monkeypatch):
    """With HBM already in use before the run, nothing is built or timed and
    the exit status is 3."""
    import torch

    monkeypatch.setattr(torch.cuda, "is_available", lambda: True)
    monkeypatch.setattr(torch.cuda, "set_device", lambda d: None)
    monkeypatch.setattr(bench, "check_idle",
                        lambda torch_: {"shared": True, "hbm_in_use_gib": 9.0})
    built = []
    monkeypatch.setattr(bench, "trajectory_leg", lambda *a: built.append(a))
    args = bench.argparse.Namespace(allow_shared_gpu=False)
    assert bench.run_legs(args, ["trajectory"]) == 3
    assert built == []


def test_shared_threshold_is_applied(monkeypatch):
    class Cuda:
        @staticmethod
        def mem_get_info():
            return (100 << 30, 288 << 30)

        @staticmethod
        def memory_reserved():
            return 0

    class FakeTorch:
        cuda = Cuda

    monkeypatch.setenv("ROCPROF_FAKE", "1")  # skips the rocm-smi query
    st = bench.check_idle(FakeTorch)
    assert st["shared"] and st["hbm_in_use_gib"] == pytest.approx(188.0)
