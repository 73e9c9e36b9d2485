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
    # the fused op-count floors per 64-byte block; MD5 needs no byte-order perms on the
    # dword-aligned fixed-length batches the roofline is quoted on
    assert bench.OPS_PER_BLOCK == {"md5": 324, "sha1": 613, "sm3": 1348}
    # the same counts split into full-rate (2 cycles per wave64 instruction) and half-rate
    # (4 cycles) ops, and the peak each mix gives at 1,024 SIMDs x 2.4 GHz
    for a, (full, half) in bench.OPS_BY_RATE.items():
        assert full + half == bench.OPS_PER_BLOCK[a]
        want = bench.OPS_PER_BLOCK[a] * 64 * 1024 * 2.4e9 / (2 * full + 4 * half) / 1e12
        assert abs(bench.ALU_PEAK_MIX_TOPS[a] - want) < 1e-9
    assert abs(bench.ALU_PEAK_MIX_TOPS["sm3"] - 47.93) < 0.01 and abs(bench.ALU_PEAK_MIX_TOPS["md5"] - 56.37) < 0.01


def test_critical_path_bound():
    import numpy as np

    sys.path.insert(0, str(ROOT))
    import bench

    lens = np.array([1 << 20, 100], np.uint64)
    # 16,385 blocks x 1,348 ops x 4 cycles at 2.1 GHz
    got = bench._critical_path_ms(lens, np.array([2, 0], np.uint8), None, clock_ghz=2.1)
    assert abs(got - 16385 * 1348 * 4 / 2.1e9 * 1e3) < 1e-9


def test_rounds_only_critical_path():
    import numpy as np

    sys.path.insert(0, str(ROOT))
    import bench

    lens = np.array([1 << 20, 1 << 19], np.uint64)
    got = bench._critical_path_ms(lens, np.array([2, 1], np.uint8), None, per_block=bench.ROUNDS_ONLY_OPS)
    assert abs(got - 16385 * 921 * 4 / 2.1e9 * 1e3) < 1e-9


def test_record_traffic_scales_by_the_copy_kernel(tmp_path, monkeypatch):
    """Counter CSVs of two runs -> bytes per launch: each counter scaled by the factor that
    makes the largest copy-kernel dispatch read (write) exactly 1 GiB."""
    sys.path.insert(0, str(ROOT))
    import bench

    def write_csv(d, rows):
        d.mkdir()
        with open(d / "x_counter_collection.csv", "w") as f:
            f.write("Kernel_Name,Counter_Value\n")
            for name, kib in rows:
                f.write(f'"{name}",{kib}\n')

    plain = "void hb::k_plain<{}, true>(unsigned char const*, unsigned long)"
    lds = "void hb::k_plain_lds<{}>(unsigned char const*, unsigned long, unsigned long, unsigned char*)"
    # the copy kernel reads 1 GiB but the counter says half of it in KiB; a small copy too.
    # The default plain kernel is the LDS-staged one; the per-lane one is the alternative
    write_csv(tmp_path / "fetch", [("__amd_rocclr_copyBuffer", 524288), ("__amd_rocclr_copyBuffer", 10),
                                   (lds.format(0), 512 * 1024), (lds.format(0), 512 * 1024),
                                   (plain.format(0), 520 * 1024),
                                   (lds.format(1), 600 * 1024), (lds.format(2), 700 * 1024)])
    write_csv(tmp_path / "write", [("__amd_rocclr_copyBuffer", 1 << 20), (lds.format(0), 16 * 1024),
                                   (plain.format(0), 16 * 1024),
                                   (lds.format(1), 20 * 1024), (lds.format(2), 32 * 1024)])
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", out)
    bench.record_traffic(str(tmp_path / "fetch"), str(tmp_path / "write"))
    t = json.loads(out.read_text())
    assert t["read_factor"] == 2.0 and t["write_factor"] == 1.0
    assert t["fixed:md5"]["fetch_bytes"] == 1 << 30 and t["fixed:md5"]["write_bytes"] == 16 << 20
    assert t["fixed:md5"]["kernel"] == "hb::k_plain_lds<0>" and t["fixed:sm3"]["kernel"] == "hb::k_plain_lds<2>"
    assert t["fixed_alt:md5"]["fetch_bytes"] == 2 * 520 * (1 << 20)
    assert "fixed_alt:sha1" not in t  # no counters for it in this run
    assert t["fixed:sm3"]["bytes_per_launch"] == 2 * 700 * (1 << 20) + (32 << 20)
    assert t["fixed:sha1"]["source_hash"] == bench.kernel_source_hash()
    monkeypatch.setattr(bench, "TRAFFIC_FILE", out)
    assert bench.measured_traffic("sm3", "fixed") == t["fixed:sm3"]["bytes_per_launch"]


def test_hw_queue_setting(monkeypatch):
    """The serving section runs with eight HIP hardware queues (`--workload serve`, or the
    full run's child process); --hw-queues sets the count for the process; with neither
    the environment's value is left alone."""
    sys.path.insert(0, str(ROOT))
    import bench

    monkeypatch.setenv("GPU_MAX_HW_QUEUES", "4")
    bench._set_hw_queues(["bench.py"])
    assert bench.os.environ["GPU_MAX_HW_QUEUES"] == "4"
    bench._set_hw_queues(["bench.py", "--workload", "serve"])
    assert bench.os.environ["GPU_MAX_HW_QUEUES"] == str(bench.SERVE_HW_QUEUES_DEFAULT) == "8"
    bench._set_hw_queues(["bench.py", "--workload=serve", "--hw-queues", "6"])
    assert bench.os.environ["GPU_MAX_HW_QUEUES"] == "6"
    bench._set_hw_queues(["bench.py", "--hw-queues=12"])
    assert bench.os.environ["GPU_MAX_HW_QUEUES"] == "12"
