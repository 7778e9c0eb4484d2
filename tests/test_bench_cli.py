"""The benchmark's command-line contract on the host: more than one GPU is
refused with a JSON error line and a non-zero exit status before any device
work; the roofline byte counts are the sums of the fields each kernel reads
and writes."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_roofline_bytes():
    sys.path.insert(0, ROOT)
    import bench
    # eps_{n+1}, a_n (6 doubles each) and the phase id in; sigma, a_{n+1} out
    assert bench.BYTES_PER_POINT == 6 * 8 + 6 * 8 + 1 + 6 * 8 + 6 * 8 == 193
    assert bench.BYTES_PER_POINT_TANGENT == 193 + 36 * 8
    # the conventional entry point also writes an int32 iteration count
    assert bench.BYTES_PER_POINT_CONVENTIONAL == 193 + 4
    # FP32: 4-byte components
    assert bench.BYTES_PER_POINT_F32 == 6 * 4 * 4 + 1
    assert bench.BYTES_PER_POINT_F32_TANGENT == 97 + 36 * 4
    # adaptive schemes: eps_n, eps_{n+1}, a_n, phase in; sigma, a_{n+1},
    # int32 step count out
    assert bench.BYTES_PER_POINT_RK == 3 * 48 + 1 + 2 * 48 + 4
    assert bench.BYTES_PER_POINT_RK_TANGENT == bench.BYTES_PER_POINT_RK + 36 * 8
    r = bench.hbm_roofline(200, 10 ** 6, 0.1)
    assert r["bound"] == "hbm" and abs(r["achieved"] - 2000.0) < 1e-9
    assert abs(r["frac"] - 2000.0 / bench.HBM_PEAK_GBS) < 1e-12
    # basic scheme on 128 x 128 planes: the half spectrum holds 6 x 128 x 65
    # complex values per plane of 128 x 128 voxels
    half = 6 * 65 * 16 / 128
    assert abs(bench.MS_HALF_SPECTRUM_BYTES - half) < 1e-12
    sweep, fwd, z, inv = 97 + 48, 48 + half, 2 * half, half + 96
    assert abs(bench.MS_BYTES_PER_VOXEL - (sweep + fwd + z + inv)) < 1e-9
    assert abs(bench.MS_BYTES_PER_VOXEL - 484.0) < 1e-9
