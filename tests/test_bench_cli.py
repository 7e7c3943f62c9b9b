"""bench.py on the CPU: the one-GPU contract and the committed traffic figures."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_figures_come_from_committed_profiles():
    import bench
    v = bench.measured_traffic("k_dc_spmv_dot<float,10>", "config2", 0)
    assert v is not None and 40e6 < v < 60e6
    # no figure for another split, another kernel or a workload without counters
    assert bench.measured_traffic("k_dc_spmv_dot<float,10>", "config2", 2048) is None
    assert bench.measured_traffic("k_dc_axpy<float,10>", "config2", 0) is None
    assert bench.measured_traffic("k_dc_spmv_dot<float,10>", "config1", 0) is None


def test_algorithmic_bytes():
    import bench
    U, S = 709620, 3
    # stencil + multi-dot of step 10 in FP32: (10 + 5) * 4 B + 16 B / 3 per unknown
    assert abs(bench.alg_bytes_active(1, 10, U, 1, S, True) - (60 + 16 / 3) * U) < 1
    # delayed-scheme axpy: 3 t at step 0, t (j + 4) after
    assert bench.alg_bytes_active(2, 0, U, 1, S, True) == 12 * U
    assert bench.alg_bytes_active(2, 10, U, 1, S, True) == 56 * U
    # CGS2 second pass, FP64: t (j + 3)
    assert bench.alg_bytes_active(2, 10, U, 0, S, False) == 8 * 13 * U


def test_unet_work_per_voxel():
    import bench
    # 16-32-64-64 U-Net, 13 inputs, 3 outputs: 40,224 multiply-adds per voxel at full
    # resolution (12,528 down, 27,648 up, 48 head), 152,064 / 8, 497,664 / 64, 221,184 / 512
    assert bench.unet_macs_per_voxel(13, 3, [16, 32, 64, 64]) == 40224 + 19008 + 7776 + 432
    # one level, no skips: two convolutions and the head
    assert bench.unet_macs_per_voxel(2, 1, [4]) == 2 * 4 * 27 + 4 * 4 * 27 + 4


def test_network_widths_option():
    import pytest

    import bench
    assert bench.net_widths(None, "16,16,16") == [16, 16, 16]
    assert bench.net_widths("16,32,64,64", "16,16,16") == [16, 32, 64, 64]
    for bad in ("32,32", "16,24", "16,16,16,16,16,16,16", "16,x", "16,,32"):
        with pytest.raises(SystemExit):
            bench.net_widths(bad, "16,16,16")
