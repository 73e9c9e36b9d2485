"""bench.py contract checks that need no GPU."""
import json
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parent.parent


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    assert rec["n_gpus"] == 2 and "one GPU" in rec["error"]


def test_roofline_constants():
    sys.path.insert(0, str(ROOT))
    import bench

    # 256 CUs x 64 lanes x 2.4 GHz
    assert abs(bench.ALU_PEAK_TOPS - 39.3216) < 1e-9
    assert bench.OPS_PER_BLOCK == {"md5": 340, "sha1": 613, "sm3": 1348}


def test_critical_path_bound():
    import numpy as np

    sys.path.insert(0, str(ROOT))
    import bench

    lens = np.array([1 << 20, 100], np.uint64)
    # 16,385 blocks x 1,348 ops x 4 cycles at 2.1 GHz
    got = bench._critical_path_ms(lens, np.array([2, 0], np.uint8), None, clock_ghz=2.1)
    assert abs(got - 16385 * 1348 * 4 / 2.1e9 * 1e3) < 1e-9
