#!/usr/bin/env python3
"""Benchmark of MI355X batch hashing (MD5, SHA-1, SM3).

Default workload: each of MD5, SHA-1 and SM3 over 2^20 messages of exactly 1,024 bytes
(16 blocks + a padding block each), uniform random bytes, one contiguous device buffer,
digests out.  One step hashes the whole buffer with all three algorithms (three plain
launches); inputs are resident in HBM before timing starts.

    python bench.py [--steps K] [--warmup W] [--workload fixed|uneven|mixed|serve]

Prints ONE JSON line.  `value` is hashed GB/s (10^9 bytes of message payload per second)
over the timed steps; per-algorithm kernel times come from HIP events recorded on the
stream the kernels run on; `roofline` is reported for the dominant (slowest) kernel;
`cpu_baseline` times the CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from pathlib import Path

import numpy as np

# Hardware queues per process for HIP (GPU_MAX_HW_QUEUES, read once when the runtime
# starts).  The serving loop wants eight rather than HIP's four, so it can run two
# long-chain streams and two copy streams beside its short-chain stream and the process's
# own default stream without two of them sharing a queue; the batched mixed plan runs best
# with the default four.  So the full run measures serving first, in a child process
# started with --serve-hw-queues (default 8) before this process touches the GPU;
# `--workload serve` alone uses 8, and --hw-queues sets the value for this process.  Set here, before anything initialises the GPU; the values used
# are reported in the output line.
SERVE_HW_QUEUES_DEFAULT = 8


def _set_hw_queues(argv):
    n = None
    for i, a in enumerate(argv):
        if a == "--hw-queues" and i + 1 < len(argv):
            n = int(argv[i + 1])
        elif a.startswith("--hw-queues="):
            n = int(a.split("=", 1)[1])
    if n is None and ("--workload=serve" in argv or ("serve" in argv and "--workload" in argv)):
        n = SERVE_HW_QUEUES_DEFAULT
    if n is not None:
        os.environ["GPU_MAX_HW_QUEUES"] = str(n)


_set_hw_queues(sys.argv)

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

ALGO_NAMES = ["md5", "sha1", "sm3"]
# VALU instructions per 64-byte block on gfx950 (one lane): the compression with every
# three-input boolean function as one v_bitop3_b32, rotates as v_alignbit_b32 and sums as
# v_add3_u32 / v_xad_u32, plus, for SHA-1 and SM3, one v_perm_b32 per message word for the
# byte order.  MD5's words are little-endian as loaded, so on dword-aligned messages (the
# fixed-length batches) it needs none: 64 steps x 5 + 4.
OPS_PER_BLOCK = {"md5": 324, "sha1": 613, "sm3": 1348}
# The same count split by issue rate: (full-rate, half-rate).  A gfx950 SIMD issues a wave64
# VALU instruction in 2 cycles for the plain 32-bit ops used here (v_bitop3_b32, VOP2
# v_add_u32 / v_xor_b32: 32 lanes per clock, the rate behind the 157.3 TFLOP/s fp32 vector
# peak) and in 4 cycles for the others (v_add3_u32, v_xad_u32, v_alignbit_b32, v_perm_b32).
#   MD5   per step F, + T, + b (full); add3, rotate (half); 4 final adds (full)
#   SHA-1 per round f (full); two add3, two rotates (half); per schedule word xor3, xor
#         (full), rotate (half); 5 final adds (full); 16 perms (half)
#   SM3   per round FF, GG, P0's xor3, two adds (full); two add3, two xad, six rotates
#         (half); per expansion word three xor3 (full), four rotates (half); 8 final xors
#         (full); 16 perms (half)
OPS_BY_RATE = {"md5": (196, 128), "sha1": (213, 400), "sm3": (484, 864)}
CUS, SIMDS_PER_CU, LANES, CLOCK_GHZ = 256, 4, 64, 2.4
# one lane-op per lane per clock (the half-rate class's peak): 39.32 T int32 lane-ops/s
ALU_PEAK_TOPS = CUS * LANES * CLOCK_GHZ * 1e9 / 1e12


def mix_peak_tops(name):
    """Peak lane-op rate for an algorithm's op mix from the unit counts and the clock: every
    SIMD issuing its full-rate ops in 2 cycles and its half-rate ops in 4 (wave64), no gaps."""
    full, half = OPS_BY_RATE[name]
    cycles = 2 * full + 4 * half  # per wave and block, on one SIMD
    return OPS_PER_BLOCK[name] * LANES * CUS * SIMDS_PER_CU * CLOCK_GHZ * 1e9 / cycles / 1e12


ALU_PEAK_MIX_TOPS = {a: mix_peak_tops(a) for a in OPS_PER_BLOCK}  # MD5 56.37, SHA-1 47.59, SM3 47.93
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = ROOT / "profiles" / "traffic.json"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="fixed",
                   choices=["fixed", "uneven", "mixed", "serve", "digits9", "ingest", "incremental", "valu"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=12.0, help="target oracle time in total")
    p.add_argument("--only-headline", action="store_true",
                   help="skip the batched, mixed and serving sections of the default run")
    p.add_argument("--serve-seconds", type=float, default=15.0,
                   help="offered-load time shared by the sweep's other points (0.5 C, 0.9 C, fixed rate)")
    p.add_argument("--serve-headline-seconds", type=float, default=20.0,
                   help="offered-load time of the headline point (0.7 C)")
    p.add_argument("--no-overload", action="store_true", help="skip the serving overload burst")
    p.add_argument("--save-inputs", default=None, metavar="DIR",
                   help="also write the seeded length / algorithm arrays of each section as .npy files")
    p.add_argument("--hw-queues", type=int, default=None,
                   help="HIP hardware queues for this process (GPU_MAX_HW_QUEUES, at most 32); "
                        "default: the environment's (HIP's four), eight for --workload serve")
    p.add_argument("--serve-mode", choices=("steps", "resident"), default=None,
                   help="serving loop mode (HB_SERVER_MODE): device steps per batch, or one resident "
                        "serving kernel that requests join; default: the library's")
    p.add_argument("--serve-hw-queues", type=int, default=SERVE_HW_QUEUES_DEFAULT,
                   help="hardware queues of the child process that measures serving in the full run")
    p.add_argument("--copy-calibration", action="store_true",
                   help="also run one plain 1 GiB device-to-device copy (reference for HBM counters)")
    p.add_argument("--record-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                   help="write profiles/traffic.json from the counter CSVs of two rocprofv3 runs of "
                        "--only-headline --copy-calibration (--pmc FETCH_SIZE, then --pmc WRITE_SIZE) and exit")
    return p.parse_args()


def kernel_source_hash() -> str:
    """Hash of the sources the plain kernels are built from (the roofline kernel)."""
    h = hashlib.sha256()
    for f in ("hb_device.hpp", "hb_kernels.hip"):
        h.update((ROOT / "paper_2407_09333_amd" / "csrc" / f).read_bytes())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from rocprofv3 FETCH_SIZE/WRITE_SIZE runs, if they were taken
    on the current kernel source."""
    if not TRAFFIC_FILE.exists():
        return None
    try:
        t = json.loads(TRAFFIC_FILE.read_text())
    except Exception:
        return None
    ent = t.get(f"{workload}:{kernel}")
    if not ent or ent.get("source_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def record_traffic(fetch_dir: str, write_dir: str):
    """HBM bytes per launch of the plain fixed-length kernels from rocprofv3 counter CSVs.
    Each counter is scaled by the factor that makes it read 1 GiB for the plain 1 GiB copy
    kernel of the same run (the largest __amd_rocclr_copyBuffer dispatch)."""
    import csv

    def per_kernel(d):
        f = next(Path(d).rglob("*counter_collection.csv"))
        by = {}
        for r in csv.DictReader(open(f)):
            by.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024)
        return by

    fetch, write = per_kernel(fetch_dir), per_kernel(write_dir)
    copy_f = max(v for k, vs in fetch.items() if "copyBuffer" in k for v in vs)
    copy_w = max(v for k, vs in write.items() if "copyBuffer" in k for v in vs)
    rf, wf = round((1 << 30) / copy_f, 3), round((1 << 30) / copy_w, 3)
    out = {"_about": "HBM bytes per launch of the plain fixed-length kernels on 2^20 x 1,024 B, from two "
                     "rocprofv3 runs (--pmc FETCH_SIZE, then --pmc WRITE_SIZE) of `python3 bench.py "
                     "--only-headline --no-cpu-baseline --steps 3 --warmup 1 --copy-calibration`, written by "
                     "`python3 bench.py --record-traffic FETCH_DIR WRITE_DIR`; each counter scaled by the factor "
                     "that makes it read 1 GiB for the plain 1 GiB copy kernel of that run "
                     "(__amd_rocclr_copyBuffer). source_hash = hash of hb_device.hpp and hb_kernels.hip when "
                     "the counters were taken.",
           "read_factor": rf, "write_factor": wf}
    for a, name in enumerate(ALGO_NAMES):
        # the default plain kernel (LDS-staged) and the alternative (per lane)
        kernels = {"fixed": f"hb::k_plain_lds<{a}>", "fixed_alt": f"hb::k_plain<{a}, true>"}
        for key, kname in kernels.items():
            k = next((k for k in fetch if kname in k), None)
            if k is None or k not in write:
                continue
            fb = sum(fetch[k]) / len(fetch[k]) * rf
            wb = sum(write[k]) / len(write[k]) * wf
            out[f"{key}:{name}"] = {"kernel": kname, "fetch_bytes": round(fb), "write_bytes": round(wb),
                                    "source_hash": kernel_source_hash(), "bytes_per_launch": round(fb + wb),
                                    "read_over_payload": round(fb / (1 << 30), 3)}
    TRAFFIC_FILE.write_text(json.dumps(out, indent=1) + "\n")
    print(json.dumps(out, indent=1))


def cpu_baseline_fixed(msgs_dev, n, L, target_s, gpu_digests=None):
    """The oracle on the first messages of the same buffer: all host cores (the reported
    value), and one core on a smaller sample, per algorithm.  With gpu_digests (algorithm ->
    (n, digest size) host array of the timed launches' output) every one of those digests is
    also checked against the oracle's over the whole buffer (untimed; a mismatch raises)."""
    import oracle

    cores = len(os.sched_getaffinity(0))
    verified = None
    if gpu_digests is not None:
        whole = msgs_dev[: n * L].cpu().numpy()
        offs = np.arange(n, dtype=np.uint64) * np.uint64(L)
        lens = np.full(n, L, np.uint64)
        t0 = time.perf_counter()
        for a, got in gpu_digests.items():
            want = oracle.hash_batch(a, whole, offs, lens, threads=cores)
            bad = np.flatnonzero((want != got).any(axis=1))
            if bad.size:
                raise RuntimeError(f"{ALGO_NAMES[a]}: {bad.size} of {n} digests differ from the oracle "
                                   f"(first at message {int(bad[0])})")
        verified = {"messages": n * len(gpu_digests), "all_equal_to_oracle": True,
                    "what": "every digest of the timed launches (each algorithm's default plain kernel) against "
                            "the oracle over the whole buffer; the alternative plain kernel's digests are compared "
                            "with these on the GPU",
                    "seconds": round(time.perf_counter() - t0, 2)}
        del whole
    host = msgs_dev[: min(n, 1 << 16) * L].cpu().numpy()

    def timed(a, m, threads):
        offs = np.arange(m, dtype=np.uint64) * np.uint64(L)
        lens = np.full(m, L, np.uint64)
        t0 = time.perf_counter()
        oracle.hash_batch(a, host, offs, lens, threads=threads)
        return time.perf_counter() - t0

    total_bytes, total_t, counts, per_algo = 0, 0.0, {}, {}
    for a in range(3):
        # calibrate on a small sample, then size the all-core sample for ~target_s / 4 per
        # algorithm and the one-core sample for ~target_s / 12
        dt = timed(a, 2048, cores)
        m = int(min(host.size // L, max(2048, 2048 * (target_s / 4) / max(dt, 1e-6))))
        t = timed(a, m, cores)
        m1 = int(min(host.size // L, max(256, 2048 * (target_s / 12) / max(dt * cores, 1e-6))))
        t1 = timed(a, m1, 1)
        total_t += t
        total_bytes += m * L
        counts[ALGO_NAMES[a]] = m
        per_algo[ALGO_NAMES[a]] = {"all_cores_GBps": round(m * L / t / 1e9, 3),
                                   "one_core_GBps": round(m1 * L / t1 / 1e9, 3), "one_core_messages": m1}
    return {"value": total_bytes / total_t / 1e9, "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": f"first {counts} messages of {L} B of the same buffer, per algorithm, "
                      f"plain C oracle with OpenMP over {cores} threads",
            "per_algo": per_algo, "digests_verified": verified,
            "paper_context": "the paper reports only ratios: its best CPU+GPU split over OpenSSL with OpenMP "
                             "on all CPU threads, SHA-1 55.8x, MD5 1.2x, SM3 22.5x (Sec. V-B, other "
                             "hardware and baseline); per_algo here is the plain C oracle"}


def bench_valu_probe():
    """The integer-VALU issue rates the roofline's peak rests on (hb_probe_valu): SIMD cycles
    per wave instruction for each instruction kind and two mixes, and per wave and 64-byte
    block for each algorithm's compression from registers, at 1, 4 and 8 waves per SIMD (one
    wave alone shows a lone chain's issue limit); beside them the op-mix model (2 cycles per
    full-rate op, 4 per half-rate op) and the fraction of it each compression reaches."""
    from paper_2407_09333_amd import hb

    out = {"unit": "SIMD cycles per wave instruction (md5/sha1/sm3: per wave and 64-byte block)"}
    for wps in (1, 4, 8):
        out[f"waves_per_simd_{wps}"] = {}
        for k in hb.PROBE_KINDS:
            c, g = hb.probe_valu(k, wps)
            out[f"waves_per_simd_{wps}"][k] = {"cycles": round(c, 3), "clock_ghz": round(g, 3)}
    model = {a: 2 * f + 4 * h for a, (f, h) in OPS_BY_RATE.items()}
    out["mix_model_cycles_per_block"] = model
    out["compression_frac_of_mix_peak_at_4_waves"] = {
        a: round(model[a] / out["waves_per_simd_4"][a]["cycles"], 3) for a in ALGO_NAMES}
    return out


def bench_fixed(args):
    import torch

    from paper_2407_09333_amd import hb, workloads

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    info = hb.device_info()
    n, L = 1 << 20, 1024
    b = workloads.cfg_fixed_1m_x_1024(0, device="cuda", n=n)
    msgs = b.messages
    outs = {a: torch.empty((n, hb.digest_size(a)), dtype=torch.uint8, device=dev) for a in range(3)}
    stream = torch.cuda.current_stream()

    def step(evs=None):
        for a in range(3):
            if evs is not None:
                evs[a][0].record(stream)
            hb.hash_batch_fixed(a, msgs, n, L, out=outs[a], stream=stream)
            if evs is not None:
                evs[a][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.copy_calibration:
        dst = torch.empty_like(msgs)
        dst.copy_(msgs)
        torch.cuda.synchronize()
        del dst
    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_step = {ALGO_NAMES[a]: [evs[k][a][0].elapsed_time(evs[k][a][1]) for k in range(args.steps)] for a in range(3)}
    kms = {name: float(np.mean(v)) for name, v in per_step.items()}
    ms_per_step = wall * 1e3 / args.steps
    payload = n * L
    blocks = n * ((L + 8) // 64 + 1)
    per_algo = {}
    for name in ALGO_NAMES:
        t = kms[name] / 1e3
        ops = blocks * OPS_PER_BLOCK[name]
        per_algo[name] = {
            "kernel_ms": round(kms[name], 4),
            "kernel_ms_median": round(float(np.median(per_step[name])), 4),
            "kernel_ms_min": round(float(np.min(per_step[name])), 4),
            "hashed_GBps": round(payload / t / 1e9, 1),
            "alu_Tops": round(ops / t / 1e12, 2),
            "alu_frac": round(ops / t / 1e12 / ALU_PEAK_MIX_TOPS[name], 4),
            "alu_frac_one_op_per_lane_clock": round(ops / t / 1e12 / ALU_PEAK_TOPS, 4),
            "hbm_frac_payload": round(payload / t / 1e9 / HBM_PEAK_GBS, 4),
        }
    # each algorithm again with the other plain kernel (the same digests): the default is the
    # LDS-staged kernel, the alternative the per-lane one (HB_PLAIN_LDS=0)
    default_digests = {a: outs[a].clone() for a in range(3)}
    for a in range(3):
        alt = "per_lane"
        os.environ["HB_PLAIN_LDS"] = "0"
        try:
            alt_ms = []
            for k in range(args.warmup + args.steps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                hb.hash_batch_fixed(a, msgs, n, L, out=outs[a], stream=stream)
                e1.record(stream)
                e1.synchronize()
                if k >= args.warmup:
                    alt_ms.append(e0.elapsed_time(e1))
        finally:
            del os.environ["HB_PLAIN_LDS"]
        per_algo[ALGO_NAMES[a]]["kernel"] = "lds_staged"
        per_algo[ALGO_NAMES[a]][f"{alt}_kernel_ms"] = round(float(np.mean(alt_ms)), 4)
        per_algo[ALGO_NAMES[a]][f"{alt}_kernel_ms_min"] = round(float(np.min(alt_ms)), 4)
        if not torch.equal(outs[a], default_digests[a]):
            raise RuntimeError(f"{ALGO_NAMES[a]}: the {alt} kernel's digests differ from the default kernel's")
    dom = max(kms, key=kms.get)
    t_dom = kms[dom] / 1e3
    ops_dom = blocks * OPS_PER_BLOCK[dom]
    traffic = measured_traffic(dom, "fixed")
    roofline = {"kernel": f"k_plain_lds<{dom}>", "bound": "alu", "achieved": round(ops_dom / t_dom / 1e12, 3),
                "peak": round(ALU_PEAK_MIX_TOPS[dom], 2), "unit": "Tops/s (int32 lane-ops)",
                "frac": round(ops_dom / t_dom / 1e12 / ALU_PEAK_MIX_TOPS[dom], 4), "traffic": traffic,
                "ops_per_launch": ops_dom, "ops_per_block": OPS_PER_BLOCK[dom], "blocks_per_launch": blocks,
                "ops_per_block_full_half_rate": list(OPS_BY_RATE[dom]),
                "peak_note": "peak for the algorithm's op mix: full-rate ops (bitop3, VOP2 add/xor) 2 cycles, "
                             "half-rate ops (add3, xad, alignbit, perm) 4 cycles per wave64 instruction per SIMD, "
                             "1,024 SIMDs at 2.4 GHz",
                "peak_one_op_per_lane_clock": round(ALU_PEAK_TOPS, 2),
                "frac_one_op_per_lane_clock": round(ops_dom / t_dom / 1e12 / ALU_PEAK_TOPS, 4)}
    rec = {
        "metric": "hashed GB/s per algo (MD5/SHA-1/SM3), % int-VALU peak; serving p99 ms",
        "value": round(3 * payload / (ms_per_step / 1e3) / 1e9, 1),
        "unit": "GB/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "MD5, SHA-1 and SM3 each over 2^20 messages of 1,024 B (contiguous, "
                               "uniform random bytes); one step = the three plain launches",
                   "messages": n, "msg_len": L, "payload_bytes_per_step": 3 * payload},
        "per_algo": per_algo,
        "roofline": roofline,
        "device": info,
        "kernel_source": kernel_source_hash(),
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline_fixed(msgs, n, L, args.cpu_seconds,
                                                 gpu_digests={a: default_digests[a].cpu().numpy() for a in range(3)})
        for name in ALGO_NAMES:
            rec["per_algo"][name]["over_cpu_oracle_all_cores"] = round(
                per_algo[name]["hashed_GBps"] / rec["cpu_baseline"]["per_algo"][name]["all_cores_GBps"], 1)
    return rec


def _clock_ghz_note():
    return ("peak uses the 2.4 GHz peak engine clock; under this integer load the chip was "
            "measured (GRBM_GUI_ACTIVE per XCD / kernel time) at about 2.05-2.1 GHz")


# VALU instructions per block of a chain that runs the rounds only, its schedule words
# computed beforehand off the chain (the long-chain kernel's instruction counts)
ROUNDS_ONLY_OPS = {"md5": 292, "sha1": 444, "sm3": 921}


def _critical_path_ms(lengths, algos, algo, clock_ghz=2.1, per_block=None):
    """Lower bound from the longest chain: one wave issues one VALU op per 4 cycles, so a
    message of nb blocks takes at least nb * ops * 4 / f (ops = the full compression's, or
    `per_block`)."""
    per_block = per_block or OPS_PER_BLOCK
    nb = (lengths.astype(np.int64) + 8) // 64 + 1
    if algos is None:
        cost = nb * per_block[ALGO_NAMES[algo]]
    else:
        ops = np.array([per_block[a] for a in ALGO_NAMES])
        cost = nb * ops[algos]
    return float(cost.max()) * 4 / (clock_ghz * 1e9) * 1e3


def _time_stats(fn, steps, warmup, stream):
    """Mean over `steps` back-to-back runs (events around all of them), and the median and
    min of per-run event pairs, in ms."""
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    mean = e0.elapsed_time(e1) / steps
    per = []
    for _ in range(steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        per.append(a.elapsed_time(b))
    return {"mean": mean, "median": float(np.median(per)), "min": float(np.min(per))}


def _time_ms(fn, steps, warmup, stream):
    return _time_stats(fn, steps, warmup, stream)["mean"]


def _inputs_record(args, name, **arrays):
    """Provenance of a section's seeded inputs: numpy's version and each length / algorithm
    array's SHA-256 (the bytes are regenerated from the seeds in workloads.py); with
    --save-inputs DIR the arrays are also written there as .npy files."""
    rec = {"numpy": np.__version__, "generator": "paper_2407_09333_amd.workloads",
           "sha256": {k: hashlib.sha256(np.ascontiguousarray(v).tobytes()).hexdigest() for k, v in arrays.items()}}
    out_dir = getattr(args, "save_inputs", None)
    if out_dir:
        d = Path(out_dir)
        d.mkdir(parents=True, exist_ok=True)
        for k, v in arrays.items():
            np.save(d / f"{name}_{k}.npy", np.ascontiguousarray(v), allow_pickle=False)
        rec["saved_to"] = str(d)
    return rec


def bench_uneven(args, steps=5, warmup=2):
    """SM3 over 2^22 messages with lengths uniform on 0..4096 bytes, packed: the bucketed
    persistent plan (hipGraph) against the plain one-lane-per-message kernel."""
    import torch

    from paper_2407_09333_amd import hb, workloads

    b = workloads.cfg_sm3_uneven(device="cuda")
    offs, lens = hb._dev_i64(b.offsets), hb._dev_i64(b.lengths)
    out = torch.empty((b.n, 32), dtype=torch.uint8, device="cuda")
    out_d, out_p = torch.empty_like(out), torch.empty_like(out)
    stream = torch.cuda.current_stream()
    plan = hb.Plan(b.n, flags=hb.PLAN_GRAPH | hb.PLAN_AUTOTUNE)
    st_plan = _time_stats(lambda: plan.run(b.messages, offs, lens, algo=2, out=out), steps, warmup, stream)
    t_plan = st_plan["mean"]
    plan_e = hb.Plan(b.n, flags=0)
    cfg = plan.config()
    plan_e.set_config(cfg["waves_per_cu"], cfg["msgs_per_lane"], cfg["variant"])
    _time_ms(lambda: plan_e.run(b.messages, offs, lens, algo=2, out=out_d), steps, 1, stream)
    same_eager = bool(torch.equal(out_d, out))
    k_ms = plan_e.kernel_ms()
    # the same plan at the untuned defaults (16 waves per CU, one message per lane, default
    # bursts), to state what the autotuner's choice gains
    plan_d = hb.Plan(b.n, flags=hb.PLAN_GRAPH)
    t_default = _time_ms(lambda: plan_d.run(b.messages, offs, lens, algo=2, out=out_d), steps, 1, stream)
    same_default = bool(torch.equal(out_d, out))
    default_cfg = plan_d.config()
    plan_d.close()
    t_plain = _time_ms(lambda: hb.hash_batch(2, b.messages, offs, lens, out=out_p), steps, warmup, stream)
    same_plain = bool(torch.equal(out_p, out))
    if not (same_eager and same_default and same_plain):
        raise RuntimeError(f"batched uneven: digests differ (eager plan {same_eager}, untuned plan "
                           f"{same_default}, plain {same_plain})")
    payload = int(b.lengths.sum())
    blocks = int(((b.lengths.astype(np.int64) + 8) // 64 + 1).sum())
    ops = blocks * OPS_PER_BLOCK["sm3"]
    res = {
        "workload": "SM3 over 2^22 messages, lengths uniform on 0..4096 B, packed (u64 offsets/lengths)",
        "payload_bytes": payload, "blocks": blocks,
        "batched_ms": round(t_plan, 3), "batched_ms_median": round(st_plan["median"], 3),
        "batched_ms_min": round(st_plan["min"], 3), "batched_GBps": round(payload / t_plan / 1e6, 1),
        "batched_hash_kernel_ms": round(k_ms, 3),
        "plain_ms": round(t_plain, 3), "plain_GBps": round(payload / t_plain / 1e6, 1),
        "speedup_vs_plain": round(t_plain / t_plan, 3),
        "alu_frac_batched_kernel": round(ops / (k_ms / 1e3) / 1e12 / ALU_PEAK_MIX_TOPS["sm3"], 4),
        "alu_frac_plain": round(ops / (t_plain / 1e3) / 1e12 / ALU_PEAK_MIX_TOPS["sm3"], 4),
        "alu_frac_batched_kernel_one_op_per_lane_clock": round(ops / (k_ms / 1e3) / 1e12 / ALU_PEAK_TOPS, 4),
        "critical_path_ms_bound": round(_critical_path_ms(b.lengths, None, 2), 3),
        "plan_config": cfg,
        "plan_config_note": "autotuned: waves per CU x messages per lane x load scheme (variant 0 default "
                            "bursts, 1 next-block prefetch, 2 one block per load, 3 two-block and 4 "
                            "four-block bursts), timed on this batch",
        "untuned_config": default_cfg, "untuned_ms": round(t_default, 3),
        "autotune_gain": round(t_default / t_plan, 3),
        "digests_equal_plain": same_plain,
        "inputs": _inputs_record(args, "sm3_uneven", lengths=b.lengths),
    }
    plan.close()
    plan_e.close()
    del b, offs, lens, out, out_d, out_p
    torch.cuda.empty_cache()
    return res


def bench_mixed(args, steps=3, warmup=1):
    """8 GiB, algorithm uniform per message, log-normal lengths (median 512 B, sigma 1.5,
    cap 1 MiB): one fused persistent launch in a hipGraph against one plain launch per
    algorithm."""
    import torch

    from paper_2407_09333_amd import hb, workloads

    b = workloads.cfg_mixed_8gib(device="cuda")
    offs, lens, al = hb._dev_i64(b.offsets), hb._dev_i64(b.lengths), hb._dev_u8(b.algos)
    out = torch.empty((b.n, 32), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    plan = hb.Plan(b.n, flags=hb.PLAN_GRAPH)
    st_plan = _time_stats(lambda: plan.run(b.messages, offs, lens, algos=al, out=out), steps, warmup, stream)
    t_plan = st_plan["mean"]
    out_p = torch.empty_like(out)
    t_plain = _time_ms(lambda: hb.hash_batch_mixed(al, b.messages, offs, lens, out=out_p), steps, warmup, stream)
    same_plain = bool(torch.equal(out_p, out))
    if not same_plain:
        raise RuntimeError("batched mixed: the fused plan's digests differ from the plain launches'")
    payload = int(b.lengths.sum())
    nb = (b.lengths.astype(np.int64) + 8) // 64 + 1
    ops = int((nb * np.array([OPS_PER_BLOCK[a] for a in ALGO_NAMES])[b.algos]).sum())
    # the throughput bound: each algorithm's ops at its own mix peak
    t_peak_s = float(sum((nb[b.algos == k].sum() * OPS_PER_BLOCK[a]) / (ALU_PEAK_MIX_TOPS[a] * 1e12)
                         for k, a in enumerate(ALGO_NAMES)))
    cp = _critical_path_ms(b.lengths, b.algos, None)
    cp_ro = _critical_path_ms(b.lengths, b.algos, None, per_block=ROUNDS_ONLY_OPS)
    res = {
        "workload": "8 GiB mixed MD5/SHA-1/SM3 per message, log-normal lengths (median 512 B, sigma 1.5, "
                    "cap 1 MiB), packed",
        "messages": b.n, "payload_bytes": payload, "max_len": int(b.lengths.max()),
        "fused_ms": round(t_plan, 3), "fused_ms_median": round(st_plan["median"], 3),
        "fused_ms_min": round(st_plan["min"], 3), "fused_GBps": round(payload / t_plan / 1e6, 1),
        "plain_3_launches_ms": round(t_plain, 3), "plain_GBps": round(payload / t_plain / 1e6, 1),
        "speedup_vs_plain": round(t_plain / t_plan, 3),
        "throughput_bound_ms": round(t_peak_s * 1e3, 3),
        "critical_path_ms_full_compression": round(cp, 3),
        "critical_path_ms_bound": round(cp_ro, 3),
        "frac_of_critical_path_bound": round(cp_ro / t_plan, 4),
        "critical_path_note": "longest chain x ops per block x 4 cycles at 2.1 GHz; the bound uses the "
                              "rounds-only chain (schedule words precomputed off the chain), the other "
                              "figure the full compression",
        "digests_equal_plain": same_plain,
        "inputs": _inputs_record(args, "mixed_8gib", lengths=b.lengths, algos=b.algos),
    }
    plan.close()
    del b, offs, lens, al, out, out_p
    torch.cuda.empty_cache()
    return res


def bench_ingest(args, reps=3):
    """Host-resident input (the ingest row): SM3 over 2^20 messages with lengths uniform on
    0..4096 B (about 2.15 GB) in pageable host memory.  hash_batch_host (chunked H2D on a
    copy stream overlapped with hashing) against copying everything first (pageable H2D,
    then the plan), and against the same plan on device-resident input (kernel-only)."""
    import torch

    from paper_2407_09333_amd import hb, workloads

    b = workloads.uniform_lengths_batch(2, 1 << 20, 4096, seed=3)
    payload = int(b.lengths.sum())
    hb.hash_batch_host(b.messages[: 1 << 20], b.offsets[:100], b.lengths[:100] * 0, algo=2)  # warm buffers
    hb.hash_batch_host(b.messages, b.offsets, b.lengths, algo=2, chunk_bytes=64 << 20)
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        hb.hash_batch_host(b.messages, b.offsets, b.lengths, algo=2, chunk_bytes=64 << 20)
        ts.append(time.perf_counter() - t0)
    t_overlap = min(ts)
    plan = hb.Plan(b.n, flags=hb.PLAN_GRAPH)
    offs, lens = hb._dev_i64(b.offsets), hb._dev_i64(b.lengths)
    host = torch.from_numpy(b.messages)
    dev = host.cuda()
    plan.run(dev, offs, lens, algo=2)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        dev = host.cuda()
        plan.run(dev, offs, lens, algo=2)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    t_seq = min(ts)
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        plan.run(dev, offs, lens, algo=2)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    t_dev = min(ts)
    plan.close()
    return {"workload": "SM3, 2^20 messages, lengths uniform on 0..4096 B, packed, in pageable host memory",
            "payload_bytes": payload,
            "overlapped_end_to_end_GBps": round(payload / t_overlap / 1e9, 2),
            "copy_then_hash_GBps": round(payload / t_seq / 1e9, 2),
            "device_resident_GBps": round(payload / t_dev / 1e9, 1),
            "small_batches": bench_small_host_batches(),
            "cpu_gpu_split": bench_duty_ratio(b, t_overlap),
            "note": "end-to-end rates include the host-to-device link and host copies; not the headline value"}


def bench_duty_ratio(b, t_gpu, reps=3):
    """The CPU + GPU split of Sec. V-D on the ingest batch (SM3, host-resident): the host
    share's rate on its own, the fraction x* that Eq. 1-3 predict from the two rates
    (T_cpu(x) = T_gpu(x) with T_cpu = x S / r_cpu and T_gpu = (1 - x) S / r_gpu), and a sweep
    of x in steps of 0.02 as in Sec. V-C.  Host threads for the CPU share: half of the
    process's cores, the other half packing the GPU share's chunks."""
    from paper_2407_09333_amd import hb

    payload = int(b.lengths.sum())
    threads = max(1, len(os.sched_getaffinity(0)) // 2)
    m = 1 << 16
    hb.cpu_hash_batch(b.messages, b.offsets[:1024], b.lengths[:1024], algo=2, threads=threads)
    t0 = time.perf_counter()
    hb.cpu_hash_batch(b.messages, b.offsets[:m], b.lengths[:m], algo=2, threads=threads)
    r_cpu = int(b.lengths[:m].sum()) / (time.perf_counter() - t0)
    r_gpu = payload / t_gpu
    x_pred = r_cpu / (r_cpu + r_gpu)
    sweep = []
    for k in range(11):
        x = 0.02 * k
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            hb.hash_batch_host_split(b.messages, b.offsets, b.lengths, algo=2, cpu_fraction=x, cpu_threads=threads)
            ts.append(time.perf_counter() - t0)
        sweep.append({"x": round(x, 2), "ms": round(min(ts) * 1e3, 2), "GBps": round(payload / min(ts) / 1e9, 2)})
    best = min(sweep, key=lambda r: r["ms"])
    return {"cpu_threads": threads, "cpu_share_GBps": round(r_cpu / 1e9, 3), "gpu_path_GBps": round(r_gpu / 1e9, 2),
            "predicted_x": round(x_pred, 4), "sweep": sweep, "best_x": best["x"], "best_GBps": best["GBps"],
            "gain_vs_gpu_only": round(sweep[0]["ms"] / best["ms"], 3)}


def bench_small_host_batches(reps=30):
    """Latency of hash_batch_host on small batches: hashed in place from pinned memory
    (zero-copy) against the copy-engine path (HB_HOST_ZERO_COPY_MAX=0), median of reps
    calls, microseconds.  Cases: 4,096 x 55 B MD5 (one block each) and 1 KiB messages
    (64 KiB .. 64 MiB of payload) with MD5 and SM3."""
    from paper_2407_09333_amd import hb, workloads

    cases = [("md5 4096 x 55 B", 0, 4096, 55)]
    for n in (64, 1024, 4096, 16384, 65536):
        for a, name in ((0, "md5"), (2, "sm3")):
            cases.append((f"{name} {n} x 1 KiB", a, n, 1024))
    res = {}
    old = os.environ.get("HB_HOST_ZERO_COPY_MAX")
    try:
        for label, a, n, L in cases:
            msgs = workloads.host_random_bytes(n * L, seed=1)
            offs = np.arange(n, dtype=np.uint64) * np.uint64(L)
            lens = np.full(n, L, np.uint64)
            row = {}
            for mode, env in (("zero_copy_us", str(1 << 40)), ("copy_engine_us", "0")):
                os.environ["HB_HOST_ZERO_COPY_MAX"] = env
                hb.hash_batch_host(msgs, offs, lens, algo=a)
                ts = []
                for _ in range(reps):
                    t0 = time.perf_counter()
                    hb.hash_batch_host(msgs, offs, lens, algo=a)
                    ts.append(time.perf_counter() - t0)
                row[mode] = round(float(np.median(ts)) * 1e6, 1)
            res[label] = row
    finally:
        if old is None:
            os.environ.pop("HB_HOST_ZERO_COPY_MAX", None)
        else:
            os.environ["HB_HOST_ZERO_COPY_MAX"] = old
    return res


def bench_incremental(args, pieces=4, steps=10, warmup=2):
    """Incremental hashing: the 2^20 x 1,024 B headline batch of each algorithm hashed in
    `pieces` pieces per message -- init, update with whole-block pieces, final with the
    last -- against one plain launch over whole messages; the pieces arrive in separate
    launches with the chaining state in device memory (48 B per message)."""
    import torch

    from paper_2407_09333_amd import hb, workloads

    n, L = 1 << 20, 1024
    b = workloads.cfg_fixed_1m_x_1024(0, device="cuda", n=n)
    stream = torch.cuda.current_stream()
    piece = L // pieces
    base = torch.arange(n, dtype=torch.int64, device="cuda") * L
    lens = torch.full((n,), piece, dtype=torch.int64, device="cuda")
    res = {"workload": f"2^20 x 1,024 B per algorithm in {pieces} pieces of {piece} B per message "
                       f"(init + {pieces - 1} updates + final), device-resident", "pieces": pieces}
    for a, name in enumerate(ALGO_NAMES):
        out = torch.empty((n, hb.digest_size(a)), dtype=torch.uint8, device="cuda")

        def run():
            st = hb.hash_init(a, n, stream=stream)
            for k in range(pieces - 1):
                hb.hash_update(a, st, b.messages, base + k * piece, lens, stream=stream)
            hb.hash_final(a, st, b.messages, base + (pieces - 1) * piece, lens, out=out, stream=stream)

        t_inc = _time_ms(run, steps, warmup, stream)
        got = out.clone()
        t_one = _time_ms(lambda: hb.hash_batch_fixed(a, b.messages, n, L, out=out, stream=stream), steps, warmup,
                         stream)
        res[name] = {"pieces_ms": round(t_inc, 4), "one_shot_ms": round(t_one, 4),
                     "pieces_GBps": round(n * L / t_inc / 1e6, 1), "overhead": round(t_inc / t_one, 3),
                     "same_digests_as_one_shot": bool(torch.equal(got, out))}
    del b
    torch.cuda.empty_cache()
    return res


def bench_digits9(args):
    """The paper's workload (Sec. V-A.2): all 10^9 nine-character decimal strings, hashed
    with each algorithm; the strings are generated on the device, digests written to HBM in
    chunks of 2^27 (the output buffer is reused)."""
    import torch

    from paper_2407_09333_amd import hb

    N, chunk = 1_000_000_000, 1 << 27
    stream = torch.cuda.current_stream()
    res = {"workload": "the 10^9 nine-character decimal strings 000000000..999999999 (9 B each), generated "
                       "on the device; one padded block per message", "messages": N}
    for a, name in enumerate(ALGO_NAMES):
        out = torch.empty((chunk, hb.digest_size(a)), dtype=torch.uint8, device="cuda")
        hb.hash_digits9(a, 0, chunk, out=out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for s0 in range(0, N, chunk):
            hb.hash_digits9(a, s0, min(chunk, N - s0), out=out, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        res[name] = {"ms": round(ms, 2), "Gmsg_per_s": round(N / ms / 1e6, 2),
                     "payload_GBps": round(9 * N / ms / 1e6, 1),
                     "in_plus_digest_GBps": round((9 + hb.digest_size(a)) * N / ms / 1e6, 1)}
        del out
    torch.cuda.empty_cache()
    return res


# where a serving request's latency goes (from its trace), reported as [p50, p99] ms each:
# the client's own lateness (its submit call returning after the scheduled arrival), wait for
# admission, wait for a staging thread, packing + copy enqueue, copy completion, wait for a
# step launch, wait for the stream / metadata, the step's hashing and digest copy, and host
# completion (digests to the caller, polling)
SERVE_PARTS = ("client_late", "admit_wait", "stager_wait", "pack", "copy", "batch_wait", "exec_wait", "exec",
               "complete")


SERVE_FIXED_RATE = 8000.0  # req/s (about 7 GB/s of payload): the headline offered load


def _serve_open_loop(srv, pool, rate, n_req, seed=105):
    """n_req requests (the pool cycled) at Poisson arrivals of the given rate; latency is
    completion time - scheduled arrival time (no coordinated omission).  A consumer thread
    takes each result as it completes (Server.collect: wait, trace into an array, release, in
    submission order), as a client would, so the run holds only the requests in flight; the
    interpreter's thread switch interval is cut to 0.1 ms meanwhile so the consumer does not
    hold up a submission.  Returns the stats of the run and each request's trace split into phases."""
    import queue
    import threading

    pool_size = len(pool)
    sizes = [int(r.lengths.sum()) for r in pool]
    arrivals = np.cumsum(np.random.default_rng(seed).exponential(1.0 / rate, size=n_req))
    sched = np.zeros(n_req)
    failure = []
    q = queue.Queue()

    tr = np.zeros((n_req, len(srv.TRACE_NAMES)))

    def consume():
        try:
            for _ in range(n_req):
                k, t = q.get()
                srv.collect(t, tr[k])
        except BaseException as e:  # surfaced by the submitting thread
            failure.append(e)

    s0 = srv.stats()
    switch = sys.getswitchinterval()
    sys.setswitchinterval(1e-4)
    consumer = threading.Thread(target=consume, daemon=True)
    consumer.start()
    start = srv.now() + 0.05
    payload = 0
    try:
        for k in range(n_req):
            r = pool[k % pool_size]
            target = start + arrivals[k]
            while True:
                d = target - srv.now()
                if d <= 0:
                    break
                if d > 0.002:
                    time.sleep(d - 0.001)
            sched[k] = target
            q.put((k, srv.submit(r.messages, r.offsets, r.lengths, algo=r.algo, algos=r.algos)))
            payload += sizes[k % pool_size]
            if failure:
                break
        consumer.join()
    finally:
        sys.setswitchinterval(switch)
    if failure:
        raise failure[0]
    tm = {name: tr[:, j] for j, name in enumerate(srv.TRACE_NAMES)}
    lat = tm["done"] - sched
    phases = np.stack([tm["admit"] - sched, tm["h2d_done"] - tm["admit"], tm["done"] - tm["h2d_done"]], 1)
    # a step may be enqueued before its inputs' copy completes (the device then waits for the
    # copy), so after stage_end the copy and the step launch run side by side: batch_wait
    # counts only the time after the copy landed until the step was enqueued, exec_wait from
    # the later of the two until the step began
    ready = np.maximum(tm["launch"], tm["h2d_done"])
    parts = np.stack([np.maximum(tm["submit"] - sched, 0.0), tm["admit"] - np.maximum(tm["submit"], sched),
                      tm["stage_begin"] - tm["admit"], tm["stage_end"] - tm["stage_begin"],
                      tm["h2d_done"] - tm["stage_end"], ready - tm["h2d_done"], tm["exec_begin"] - ready,
                      tm["exec_end"] - tm["exec_begin"], tm["done"] - tm["exec_end"]], 1)
    done_max = float(tm["done"].max())
    s1 = srv.stats()
    span = done_max - start
    return {"offered_req_per_s": round(rate, 1), "requests": n_req,
            "achieved_req_per_s": round(n_req / span, 1),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "p999_ms": round(float(np.percentile(lat, 99.9)) * 1e3, 3),
            "achieved_GBps": round(payload / span / 1e9, 3),
            "steps": s1["steps"] - s0["steps"], "admission_stalls": s1["stalls"] - s0["stalls"],
            "median_ms_queue_staging_device": [round(float(x) * 1e3, 3) for x in np.median(phases, 0)],
            "p99_ms_queue_staging_device": [round(float(x) * 1e3, 3) for x in np.percentile(phases, 99, axis=0)],
            "parts_ms": {name: [round(float(np.percentile(parts[:, j], q)) * 1e3, 3) for q in (50, 99)]
                         for j, name in enumerate(SERVE_PARTS)}}


SERVE_TRACK_FRAC = 0.97   # an offered rate is sustained if the achieved rate is at least this share of it
SERVE_P99_BOUND_MS = 10.0  # ... and p99 stays below this


def _sustained(run):
    return (run["achieved_req_per_s"] >= SERVE_TRACK_FRAC * run["offered_req_per_s"]
            and run["p99_ms"] <= SERVE_P99_BOUND_MS)


def bench_serve(args, pool_size=256, seconds=15.0, fractions=(0.5, 0.7, 0.9), cap_burst=8192, trial_s=1.5):
    """Open-loop Poisson arrivals; each request 1..10,000 messages (log-uniform count),
    algorithm uniform over the three, lengths log-normal (median 256 B, cap 64 KiB); device
    budget 64 GiB.  A saturating burst of 8,192 requests gives a first estimate C_burst
    (adjacent requests then share transfers, so it can miss what Poisson arrivals get);
    the capacity C is then the highest offered rate, found by bisection over short
    open-loop trials (from 0.25 C_burst; the bracket's upper end starts at 1.1 C_burst and
    is raised while still sustained), at which the achieved rate tracks the offered one
    (>= 97 %) with p99 <= 10 ms.  The headline is p50 / p99 at 0.7 C; the sweep
    adds 0.5 and 0.9 C and the fixed rate of 8,000 req/s."""
    from paper_2407_09333_amd import hb, workloads

    if getattr(args, "serve_mode", None):
        os.environ["HB_SERVER_MODE"] = args.serve_mode
    mode = os.environ.get("HB_SERVER_MODE", "steps")
    pool = workloads.serving_requests(pool_size, 1.0, seed=5)
    srv = hb.Server(hbm_budget_bytes=64 << 30, max_slots=1024)
    for r in pool[:16]:  # warm-up
        srv.wait(srv.submit(r.messages, r.offsets, r.lengths, algo=r.algo, algos=r.algos))
    t0 = srv.now()
    burst = [pool[k % pool_size] for k in range(cap_burst)]
    ts = [srv.submit(r.messages, r.offsets, r.lengths, algo=r.algo, algos=r.algos) for r in burst]
    for t in ts:
        srv.wait(t)
    t1 = max(srv.times(t)["done"] for t in ts)
    for t in ts:
        srv.release(t)
    burst_rps = len(burst) / (t1 - t0)
    mean_bytes = float(np.mean([int(r.lengths.sum()) for r in pool]))
    print(f"bench: serving burst capacity {burst_rps:.0f} req/s", file=sys.stderr, flush=True)
    # open-loop capacity: bracket it (from 0.25 C_burst up, the upper end raised by 1.5x
    # while it is still sustained, at most three times), then bisect
    trials = []

    def trial(rate, seed):
        run = _serve_open_loop(srv, pool, rate, int(max(rate * trial_s, 300)), seed=seed)
        trials.append(run)
        print(f"bench: serving trial {rate:.0f} req/s: achieved {run['achieved_req_per_s']:.0f}, "
              f"p99 {run['p99_ms']} ms", file=sys.stderr, flush=True)
        return _sustained(run)

    lo = 0.25 * burst_rps
    hi = lo
    if trial(lo, 201):
        hi = 1.1 * burst_rps
        for grow in range(3):
            if not trial(hi, 210 + grow):
                break
            lo, hi = hi, 1.5 * hi
        else:
            hi = lo  # still sustained at the last bracket: C is at least lo
    for it in range(5):
        if hi <= lo * 1.03:
            break
        mid = 0.5 * (lo + hi)
        if trial(mid, 202 + it):
            lo = mid
        else:
            hi = mid
    cap_rps = lo
    runs = []
    headline_s = getattr(args, "serve_headline_seconds", 20.0)
    for frac in (0.7,) + tuple(f for f in fractions if f != 0.7) + (None,):
        rate = SERVE_FIXED_RATE if frac is None else frac * cap_rps
        if frac == 0.7:  # the headline: a long run (hundreds of thousands of requests)
            n_req = int(min(max(rate * headline_s, 200), 1_000_000))
        else:
            n_req = int(min(max(rate * seconds / (len(fractions) + 1), 200), 30_000))
        run = _serve_open_loop(srv, pool, rate, n_req)
        run["load_fraction"] = frac
        runs.append(run)
        where = f"{rate:.0f} req/s" if frac is None else f"{frac} C"
        print(f"bench: serving at {where}: p50 {run['p50_ms']} ms p99 {run['p99_ms']} ms",
              file=sys.stderr, flush=True)
    peak = srv.stats()["peak_bytes"]
    srv.close()
    overload = None if getattr(args, "no_overload", False) else bench_serve_overload(pool)
    head = runs[0]  # 0.7 C
    return {
        "workload": "Poisson arrivals; 1..10,000 messages per request (log-uniform), algorithm uniform, "
                    "lengths log-normal (median 256 B, sigma 1.5, cap 64 KiB); payload in host memory "
                    "(PCIe- and host-copy-inclusive); device budget 64 GiB",
        "mode": mode,
        "capacity_req_per_s": round(cap_rps, 1), "capacity_GBps": round(cap_rps * mean_bytes / 1e9, 3),
        "capacity_rule": f"highest open-loop Poisson rate with achieved >= {SERVE_TRACK_FRAC} x offered and "
                         f"p99 <= {SERVE_P99_BOUND_MS} ms (bisection over {trial_s} s trials)",
        "capacity_trials": [{k: t[k] for k in ("offered_req_per_s", "achieved_req_per_s", "p99_ms")}
                            for t in trials],
        "burst_capacity_req_per_s": round(burst_rps, 1),
        "headline": f"p50 / p99 at 0.7 C (sweep[0], {head['requests']} requests over about {headline_s:.0f} s), C the "
                    "open-loop capacity; the sweep also has 0.5 and 0.9 C and the fixed rate of "
                    f"{SERVE_FIXED_RATE:.0f} req/s (up to 30,000 requests each)",
        "offered_req_per_s": head["offered_req_per_s"], "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"],
        "p999_ms": head["p999_ms"], "achieved_GBps": head["achieved_GBps"],
        "sweep": runs, "peak_resident_bytes": peak, "overload": overload,
        "inputs": _inputs_record(args, "serving_pool",
                                 lengths=np.concatenate([r.lengths for r in pool]),
                                 algos=np.concatenate([np.full(r.lengths.size, r.algo, np.int8) if r.algos is None
                                                       else r.algos.astype(np.int8) for r in pool]),
                                 counts=np.array([r.lengths.size for r in pool], np.int64)),
    }


def bench_serve_child(args, mode=None, overload=True):
    """The serving section, measured in a child process with its own hardware-queue count
    (--serve-hw-queues), started before this process initialises the GPU; this process
    waits for it.  mode: the serving loop's mode (None: --serve-mode or the library's)."""
    import subprocess

    cmd = [sys.executable, "-u", str(Path(__file__).resolve()), "--workload", "serve",
           "--hw-queues", str(args.serve_hw_queues), "--serve-seconds", str(args.serve_seconds),
           "--serve-headline-seconds", str(args.serve_headline_seconds)]
    if args.no_overload or not overload:
        cmd.append("--no-overload")
    if args.save_inputs:
        cmd += ["--save-inputs", args.save_inputs]
    mode = mode or args.serve_mode
    if mode:
        cmd += ["--serve-mode", mode]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"serving child process failed with status {r.returncode}")
    child = json.loads(r.stdout.strip().splitlines()[-1])
    out = child["serving"]
    out["hip_hw_queues"] = child["hip_hw_queues"]
    return out


def _serve_summary(modes):
    """Both serving modes side by side: open-loop capacity, p50 / p99 at 0.7 C and at the
    fixed offered rate."""
    out = {}
    for name, sv in modes.items():
        if not sv:
            continue
        fixed = next((e for e in sv["sweep"] if e.get("load_fraction") is None), None)
        out[name] = {"capacity_req_per_s": sv["capacity_req_per_s"],
                     "p50_p99_ms_at_0.7C": [sv["p50_ms"], sv["p99_ms"]],
                     "p50_p99_ms_at_fixed_rate": [fixed["p50_ms"], fixed["p99_ms"]] if fixed else None,
                     "fixed_rate_req_per_s": SERVE_FIXED_RATE}
    return out


def bench_serve_overload(pool, n_req=160_000, budget=64 << 30):
    """Overload burst: about 140 GB of requests (the serving distribution, the pool cycled)
    submitted at once against the 64 GiB device budget, with slots enough that the budget
    is what admission waits on; every request completes, and the resident payload never
    exceeds the budget."""
    from paper_2407_09333_amd import hb

    srv = hb.Server(hbm_budget_bytes=budget, max_slots=1 << 17)
    t0 = srv.now()
    tickets, payload = [], 0
    for k in range(n_req):
        r = pool[k % len(pool)]
        tickets.append(srv.submit(r.messages, r.offsets, r.lengths, algo=r.algo, algos=r.algos))
        payload += int(r.lengths.sum())
    t_sub = srv.now() - t0
    for t in tickets:
        srv.wait(t)
        srv.release(t)
    wall = srv.now() - t0
    st = srv.stats()
    srv.close()
    res = {"requests": n_req, "payload_bytes": payload, "budget_bytes": budget, "submitted_s": round(t_sub, 3),
           "wall_s": round(wall, 3), "GBps": round(payload / wall / 1e9, 3), "completed": st["completed"],
           "admission_stalls": st["stalls"], "peak_resident_bytes": st["peak_bytes"],
           "peak_within_budget": st["peak_bytes"] <= budget}
    print(f"bench: serving overload {payload / 1e9:.1f} GB against a {budget >> 30} GiB budget: "
          f"submitted in {t_sub:.2f} s, done in {wall:.2f} s, {st['stalls']} admission stalls, "
          f"peak resident {st['peak_bytes'] / 2**30:.2f} GiB",
          file=sys.stderr, flush=True)
    return res

def main():
    args = parse()
    if args.record_traffic:
        record_traffic(*args.record_traffic)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU: messages are independent, so the path "
                                   "shards across GPUs by estimated cost with no exchange while hashing, "
                                   "and --gpus above 1 is not run",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "fixed":
        # the serving child runs first, while this process has not touched the GPU yet
        serving = None
        if not args.only_headline:
            print("bench: serving (child process)", file=sys.stderr, flush=True)
            serving = bench_serve_child(args)
            print("bench: serving, resident kernel (child process)", file=sys.stderr, flush=True)
            serving_resident = bench_serve_child(args, mode="resident", overload=False)
        rec = bench_fixed(args)
        rec["clock_note"] = _clock_ghz_note()
        if not args.only_headline:
            print("bench: batched uneven", file=sys.stderr, flush=True)
            rec["batched_uneven"] = bench_uneven(args)
            print("bench: mixed 8 GiB", file=sys.stderr, flush=True)
            rec["batched_mixed"] = bench_mixed(args)
            print("bench: ingest from host memory", file=sys.stderr, flush=True)
            rec["ingest_host_resident"] = bench_ingest(args)
            print("bench: paper workload (10^9 nine-digit strings)", file=sys.stderr, flush=True)
            rec["paper_workload_digits9"] = bench_digits9(args)
            print("bench: incremental hashing", file=sys.stderr, flush=True)
            rec["incremental"] = bench_incremental(args)
            print("bench: integer-VALU issue rates", file=sys.stderr, flush=True)
            rec["valu_issue_rates"] = bench_valu_probe()
            rec["serving"] = serving
            rec["serving_resident"] = serving_resident
            rec["serving_summary"] = _serve_summary({"steps": serving, "resident": serving_resident})
    elif args.workload == "uneven":
        rec = {"batched_uneven": bench_uneven(args, steps=args.steps, warmup=args.warmup)}
    elif args.workload == "mixed":
        rec = {"batched_mixed": bench_mixed(args, steps=args.steps, warmup=args.warmup)}
    elif args.workload == "ingest":
        rec = {"ingest_host_resident": bench_ingest(args)}
    elif args.workload == "incremental":
        rec = {"incremental": bench_incremental(args)}
    elif args.workload == "valu":
        rec = {"valu_issue_rates": bench_valu_probe()}
    elif args.workload == "digits9":
        rec = {"paper_workload_digits9": bench_digits9(args)}
    else:
        rec = {"serving": bench_serve(args, seconds=args.serve_seconds)}
    rec["hip_hw_queues"] = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
