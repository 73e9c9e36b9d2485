"""Parity of the batched form (hb_plan_*): bucketing by block count, longest-first
persistent fused launch, hipGraph replay, autotuned launch choices -- every digest
bit-exact against the CPU oracle."""
import numpy as np
import pytest

import oracle
from paper_2407_09333_amd import workloads
from tests.gpu_util import assert_same, check_guard, guarded_out, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hb():
    import torch

    assert torch.cuda.is_available()
    from paper_2407_09333_amd import hb as _hb

    return _hb


def _batch_mixed_with_long(seed=6, total=3_000_000):
    b = workloads.mixed_batch(total, seed=seed, cap=1 << 18)
    # a few long messages and empty ones among them
    rng = np.random.default_rng(seed)
    lens = b.lengths.copy()
    lens[rng.choice(b.n, 5, replace=False)] = [1 << 18, 200_000, 65_536, 0, 4095]
    offs = workloads.packed(lens)
    msgs = workloads.host_random_bytes(int(lens.sum()), seed)
    return msgs, offs, lens, b.algos


@pytest.mark.parametrize("flags", [1, 0, 4], ids=["graph", "eager", "nosort"])
@pytest.mark.parametrize("algo", [0, 1, 2])
def test_plan_single_algo_uneven(hb, flags, algo):
    b = workloads.uniform_lengths_batch(algo, 20_000, 4096, seed=13)
    print(f"case plan single algo={algo} flags={flags}", flush=True)
    plan = hb.Plan(32_768, flags=flags)
    ds = oracle.DIGEST_SIZE[algo]
    buf, out = guarded_out(b.n, ds)
    plan.run(b.messages, b.offsets, b.lengths, algo=algo, out=out)
    check_guard(buf, b.n, ds)
    assert_same(out.cpu().numpy(), oracle.hash_batch(algo, b.messages, b.offsets, b.lengths), "plan single")
    plan.close()


@pytest.mark.parametrize("flags", [1, 0], ids=["graph", "eager"])
def test_plan_mixed_with_long_empty_and_invalid(hb, flags):
    msgs, offs, lens, algos = _batch_mixed_with_long()
    al = algos.copy()
    al[::101] = 200
    print(f"case plan mixed flags={flags} n={offs.size}", flush=True)
    plan = hb.Plan(offs.size + 100, flags=flags)
    got = plan.run(msgs, offs, lens, algos=al).cpu().numpy()
    want = oracle.hash_batch(algos, msgs, offs, lens)
    want[::101] = 0
    assert_same(got, want, "plan mixed")
    plan.close()


@pytest.mark.parametrize("wpc,mpl,var", [(4, 1, 0), (8, 2, 1), (16, 4, 0), (32, 1, 1), (64, 3, 1), (16, 2, 1),
                                         (8, 1, 2), (16, 2, 2), (32, 1, 3), (16, 3, 3), (8, 2, 4), (16, 1, 4)])
def test_launch_choices_give_identical_digests(hb, wpc, mpl, var):
    """Every launch choice the autotuner may pick -- waves per CU, messages per lane and the
    message-load scheme (variant 0..4: default bursts, next-block prefetch, one block per
    load, two- and four-block bursts) -- gives the oracle's digests."""
    msgs, offs, lens, algos = _batch_mixed_with_long(seed=7, total=1_000_000)
    print(f"case choices wpc={wpc} mpl={mpl} variant={var}", flush=True)
    plan = hb.Plan(offs.size, flags=0)
    plan.set_config(waves_per_cu=wpc, msgs_per_lane=mpl, variant=var)
    cfg = plan.config()
    assert cfg["waves_per_cu"] == wpc and cfg["msgs_per_lane"] == mpl and cfg["variant"] == var
    got = plan.run(msgs, offs, lens, algos=algos).cpu().numpy()
    assert_same(got, oracle.hash_batch(algos, msgs, offs, lens), f"wpc={wpc} mpl={mpl}")
    assert plan.kernel_ms() > 0
    plan.close()


def test_set_config_rejects_unknown_scheme(hb):
    plan = hb.Plan(1000, flags=0)
    with pytest.raises(hb.HBError) as ei:
        plan.set_config(waves_per_cu=16, msgs_per_lane=1, variant=5)
    assert ei.value.status == hb.HB_EINVAL
    plan.close()


def test_autotune_cache_keyed_by_length_bucket(hb, tmp_path, monkeypatch):
    """The tuning cache file holds one line per (device, CUs, algorithm mix, length bucket):
    a fixed-length and a uniform batch of the same size and algorithm get separate lines,
    and a second plan on a batch of the same bucket reuses the cached choice."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("HB_TUNE_CACHE", str(cache))
    fixed = workloads.fixed_batch(2, 20_000, 1024, seed=51)
    unif = workloads.uniform_lengths_batch(2, 20_000, 8192, seed=52)
    cfgs = []
    for b in (fixed, unif, workloads.fixed_batch(2, 20_000, 1024, seed=53)):
        plan = hb.Plan(b.n, flags=hb.PLAN_GRAPH | hb.PLAN_AUTOTUNE)
        got = plan.run(b.messages, b.offsets, b.lengths, algo=2).cpu().numpy()
        assert_same(got, oracle.hash_batch(2, b.messages, b.offsets, b.lengths), "autotuned, bucketed cache")
        cfgs.append(plan.config())
        plan.close()
    assert cfgs[2] == cfgs[0]  # same bucket: the cached choice
    lines = [ln.split() for ln in cache.read_text().splitlines() if ln.strip()]
    buckets = {int(ln[3]) for ln in lines if ln[2] == "4"}  # algorithm mask 1 << SM3
    assert len(buckets) >= 2, lines
    assert all(int(ln[6]) in range(5) for ln in lines)


def test_autotune_picks_a_valid_choice(hb):
    b = workloads.uniform_lengths_batch(2, 30_000, 4096, seed=14)
    print("case autotune", flush=True)
    plan = hb.Plan(30_000, flags=hb.PLAN_GRAPH | hb.PLAN_AUTOTUNE)
    got = plan.run(b.messages, b.offsets, b.lengths, algo=2).cpu().numpy()
    cfg = plan.config()
    assert cfg["waves_per_cu"] in (8, 16, 32) and cfg["msgs_per_lane"] in (1, 2) and cfg["variant"] in range(5)
    assert_same(got, oracle.hash_batch(2, b.messages, b.offsets, b.lengths), "autotuned")
    plan.close()


def test_graph_replays_with_changing_inputs(hb):
    """One captured graph replayed over different batches and sizes, with eager torch work
    and synchronisations in between; every replay equals the eager (non-graph) result."""
    import torch

    plan_g = hb.Plan(50_000, flags=hb.PLAN_GRAPH)
    plan_e = hb.Plan(50_000, flags=0)
    for rep, (n, seed) in enumerate([(40_000, 1), (1_000, 2), (50_000, 3), (7, 4), (40_000, 1)]):
        print(f"case replay {rep} n={n}", flush=True)
        b = workloads.mixed_batch(n * 300, seed=seed, cap=1 << 14)
        offs, lens, al = b.offsets[:n], b.lengths[:n], b.algos[:n]
        x = torch.randn(1000, device="cuda")
        (x * 2).sum().item()  # eager work between replays
        got = plan_g.run(b.messages, offs, lens, algos=al)
        torch.cuda.synchronize()
        ref = plan_e.run(b.messages, offs, lens, algos=al)
        assert_same(got.cpu().numpy(), ref.cpu().numpy(), f"replay {rep}")
        assert_same(ref.cpu().numpy(), oracle.hash_batch(al, b.messages, offs, lens), f"eager {rep}")
    plan_g.close()
    plan_e.close()


def test_plan_rejects_oversized_batch(hb):
    plan = hb.Plan(100)
    b = workloads.uniform_lengths_batch(0, 101, 10, seed=1)
    with pytest.raises(hb.HBError) as e:
        plan.run(b.messages, b.offsets, b.lengths, algo=0)
    assert e.value.status == hb.HB_EINVAL
    plan.close()


def test_alone_equals_in_the_mix(hb):
    """Each message hashed alone by the plain kernel equals its digest from a mixed,
    bucketed batch."""
    msgs, offs, lens, algos = _batch_mixed_with_long(seed=9, total=500_000)
    print("case alone vs mix", flush=True)
    plan = hb.Plan(offs.size)
    mix = plan.run(msgs, offs, lens, algos=algos).cpu().numpy()
    for a in range(3):
        sel = np.nonzero(algos == a)[0]
        alone = hb.hash_batch(a, msgs, offs[sel], lens[sel]).cpu().numpy()
        ds = oracle.DIGEST_SIZE[a]
        assert_same(mix[sel, :ds], alone, f"alone algo {a}")
        assert not mix[sel, ds:].any()
    plan.close()


@pytest.mark.slow
def test_full_size_sm3_uneven_all(hb):
    """SM3 over 2^22 messages with lengths uniform on 0..4096 (about 8 GiB), bucketed plan
    as timed by the benchmark; every digest checked against the oracle (the whole buffer
    copied back and hashed on all host cores)."""
    import torch

    b = workloads.cfg_sm3_uneven(device="cuda")
    print(f"case full sm3 uneven n={b.n}", flush=True)
    plan = hb.Plan(b.n, flags=hb.PLAN_GRAPH)
    got = plan.run(b.messages, b.offsets, b.lengths, algo=2)
    torch.cuda.synchronize()
    _check_all(b, got, 2)
    plan.close()


@pytest.mark.slow
def test_full_size_mixed_8gib_all(hb):
    """Mixed 8 GiB batch (log-normal lengths, median 512 B, cap 1 MiB), one fused
    persistent launch as timed by the benchmark; every digest checked against the oracle."""
    import torch

    b = workloads.cfg_mixed_8gib(device="cuda")
    print(f"case full mixed n={b.n}", flush=True)
    plan = hb.Plan(b.n, flags=hb.PLAN_GRAPH)
    got = plan.run(b.messages, b.offsets, b.lengths, algos=b.algos)
    torch.cuda.synchronize()
    _check_all(b, got, b.algos)
    plan.close()


def _check_all(b, got, algo):
    host = b.messages.cpu().numpy()
    print(f"  oracle over {b.n} messages, {host.size / 1e9:.2f} GB", flush=True)
    want = oracle.hash_batch(algo, host, b.offsets, b.lengths, out_stride=got.shape[1])
    del host
    assert_same(got.cpu().numpy(), want, "full size, every digest")


def test_long_chain_direct_cap(hb, monkeypatch):
    """More long candidates than direct-chain waves (one per SIMD): a cost threshold
    across the three algorithms picks the longest chains for the long-chain kernel, the
    rest stay in the persistent kernel.  A 1 MiB scratch holds no wave of them, so every
    chosen one runs as a direct chain; on a side stream or in one launch with the bulk,
    with either persistent-kernel variant."""
    monkeypatch.setenv("HB_LONG_SCRATCH_MB", "1")
    monkeypatch.setenv("HB_LONG_MIN_BLOCKS", "2")
    rng = np.random.default_rng(41)
    n = 120_000
    lens = rng.integers(64, 1500, size=n).astype(np.uint64)
    lens[:300] = rng.integers(20_000, 90_000, size=300)
    offs = workloads.packed(lens)
    msgs = workloads.host_random_bytes(int(lens.sum()), seed=42)
    algos = rng.integers(0, 3, size=n).astype(np.uint8)
    print("case long path direct cap", flush=True)
    want = oracle.hash_batch(algos, msgs, offs, lens)
    for flags in (hb.PLAN_GRAPH, hb.PLAN_GRAPH | hb.PLAN_LONG_INLINE):
        for var in range(5):
            plan = hb.Plan(n, flags=flags)
            plan.set_config(waves_per_cu=16, msgs_per_lane=1, variant=var)
            assert_same(plan.run(msgs, offs, lens, algos=algos).cpu().numpy(), want, f"direct cap {flags} {var}")
            plan.close()


@pytest.mark.parametrize("scratch_mb,min_blocks", [("1", "256"), ("512", "2"), ("1024", "16")])
def test_long_chain_path(hb, monkeypatch, scratch_mb, min_blocks):
    """Messages above the block threshold run as rounds-only chains from precomputed
    schedule words; with a tiny scratch only some of them fit and the rest run as direct
    chains; the long-chain kernel runs beside the bulk on a side stream, or before it on
    the run's own stream.  Every digest must match the oracle either way."""
    monkeypatch.setenv("HB_LONG_SCRATCH_MB", scratch_mb)
    monkeypatch.setenv("HB_LONG_MIN_BLOCKS", min_blocks)
    rng = np.random.default_rng(int(min_blocks))
    n = 3000
    lens = rng.integers(0, 40_000, size=n).astype(np.uint64)
    lens[:40] = rng.integers(100_000, 300_000, size=40)  # some very long ones
    lens[40:50] = [0, 1, 55, 56, 63, 64, 119, 120, 16_384, 16_383]
    offs = workloads.packed(lens)
    msgs = workloads.host_random_bytes(int(lens.sum()), seed=int(min_blocks) + 1)
    algos = rng.integers(0, 3, size=n).astype(np.uint8)
    print(f"case long path scratch={scratch_mb} min_blocks={min_blocks}", flush=True)
    want = oracle.hash_batch(algos, msgs, offs, lens)
    for flags in (hb.PLAN_GRAPH, 0, hb.PLAN_GRAPH | hb.PLAN_LONG_INLINE, hb.PLAN_LONG_INLINE):
        plan = hb.Plan(n, flags=flags)
        got = plan.run(msgs, offs, lens, algos=algos).cpu().numpy()
        assert_same(got, want, f"long path flags={flags}")
        plan.close()
    plan = hb.Plan(n, flags=hb.PLAN_LONG_INLINE)
    plan.set_config(waves_per_cu=16, msgs_per_lane=2, variant=1)
    assert_same(plan.run(msgs, offs, lens, algos=algos).cpu().numpy(), want, "one launch, variant 1")
    plan.close()
    plan = hb.Plan(n, flags=hb.PLAN_NO_LONG)
    assert_same(plan.run(msgs, offs, lens, algos=algos).cpu().numpy(), want, "no long path")
    plan.close()


def _saturated_long_batch(seed=77):
    """70 SM3, 5 SHA-1 and 5 MD5 messages, every length distinct and between 1.1 and
    3 MiB -- past the ~1.05 MB point where block-count sort keys saturate -- with the
    shorter ones of each algorithm at lower indices, plus a few short messages."""
    rng = np.random.default_rng(seed)
    parts = []
    for algo, count in ((2, 70), (1, 5), (0, 5)):
        base = np.linspace(1.1 * 2**20, 3 * 2**20, count).astype(np.uint64)
        jitter = rng.permutation(count).astype(np.uint64) * np.uint64(7) + np.uint64(algo)
        parts.append((np.sort(base + jitter), np.full(count, algo, np.uint8)))
    short = rng.integers(0, 5000, size=200).astype(np.uint64)
    lens = np.concatenate([p[0] for p in parts] + [short])
    algos = np.concatenate([p[1] for p in parts] + [rng.integers(0, 3, size=200).astype(np.uint8)])
    assert np.unique(lens[:80]).size == 80
    offs = workloads.packed(lens)
    msgs = workloads.host_random_bytes(int(lens.sum()), seed)
    return msgs, offs, lens, algos


@pytest.mark.parametrize("scratch_mb", ["1024", "2048", "4096"])
def test_long_chains_past_key_saturation(hb, monkeypatch, scratch_mb):
    """Many same-algorithm messages above the saturated sort key in one plan: their order
    inside that key is arbitrary, so a long-chain wave's scratch region must hold its
    longest lane.  1 GiB holds no such wave (all run as direct chains); 2 GiB holds the
    first SM3 wave and 4 GiB both SM3 waves (rounds-only from precomputed words), the rest
    running as direct chains.  Every digest against the oracle, with the long chains beside
    the bulk on a side stream and in one launch."""
    monkeypatch.setenv("HB_LONG_SCRATCH_MB", scratch_mb)
    msgs, offs, lens, algos = _saturated_long_batch()
    print(f"case saturated long chains scratch={scratch_mb} n={lens.size}", flush=True)
    want = oracle.hash_batch(algos, msgs, offs, lens)
    for flags in (hb.PLAN_GRAPH, hb.PLAN_LONG_INLINE):
        plan = hb.Plan(lens.size, flags=flags)
        buf, out = guarded_out(lens.size, 32)
        plan.run(msgs, offs, lens, algos=algos, out=out)
        check_guard(buf, lens.size, 32)
        assert_same(out.cpu().numpy(), want, f"saturated long flags={flags} scratch={scratch_mb}")
        plan.close()
    # one algorithm per plan run too (the segment holds only saturated keys)
    sm3 = np.nonzero(algos == 2)[0]
    plan = hb.Plan(sm3.size, flags=hb.PLAN_GRAPH)
    got = plan.run(msgs, offs[sm3], lens[sm3], algo=2).cpu().numpy()
    assert_same(got, want[sm3, :32], f"saturated long sm3 only scratch={scratch_mb}")
    plan.close()


def test_long_chains_past_key_saturation_host(hb):
    """The same batch through hash_batch_host (pageable host memory, one chunk, the
    host pipeline's long-chain plan), every digest against the oracle."""
    msgs, offs, lens, algos = _saturated_long_batch(seed=78)
    print(f"case saturated long chains host n={lens.size}", flush=True)
    want = oracle.hash_batch(algos, msgs, offs, lens)
    got = hb.hash_batch_host(msgs, offs, lens, algos=algos, chunk_bytes=1 << 30)
    assert_same(got, want, "saturated long host")
