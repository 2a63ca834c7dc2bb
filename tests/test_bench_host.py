"""Host-side checks of bench.py: the one-GPU guard and the per-pair
algorithmic counts its roofline fields are computed from."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "single MI355X" in r.stderr
    assert r.stdout == ""


def test_algorithmic_counts_1mp_pair():
    # 1024 x 1024 pair, 16 x 16 windows at step 8 -> 128 x 128 nodes, +-4 px:
    # 81 shifts; per shift one multiply-add per pixel (2 flop) shared by the
    # windows holding it, 25 flop per node and shift to form and compare the
    # coefficient, 20 flop per pixel for the bilinear deformation
    a = _bench().algorithmic(1024, 1024, 128, 128, 4)
    pixels, nodes, shifts = 1 << 20, 128 * 128, 9 * 9
    assert a["corr_flop"] == 2 * shifts * pixels + 25 * shifts * nodes + 20 * pixels == 224018432
    # two u8 frames in; per node 8 B displacement, 1 B flags, 4 B vorticity, 4 B peak out
    assert a["path_bytes"] == 2 * pixels + nodes * (8 + 1 + 4 + 4) == 2375680


def test_algorithmic_counts_scale_with_radius():
    b = _bench()
    a1, a2 = b.algorithmic(512, 256, 63, 31, 1), b.algorithmic(512, 256, 63, 31, 2)
    px, nd = 512 * 256, 63 * 31
    assert a2["corr_flop"] - a1["corr_flop"] == (25 - 9) * (2 * px + 25 * nd)
    assert a1["path_bytes"] == a2["path_bytes"]
