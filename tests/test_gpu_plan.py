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


@pytest.mark.parametrize("wpc,mpl,var", [(4, 1, 0), (8, 2, 1), (16, 4, 0), (32, 1, 1), (64, 3, 1), (16, 2, 1)])
def test_launch_choices_give_identical_digests(hb, wpc, mpl, var):
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


def test_autotune_picks_a_valid_choice(hb):
    b = workloads.uniform_lengths_batch(2, 30_000, 4096, seed=14)
    print("case autotune", flush=True)
    plan = hb.Plan(30_000, flags=hb.PLAN_GRAPH | hb.PLAN_AUTOTUNE)
    got = plan.run(b.messages, b.offsets, b.lengths, algo=2).cpu().numpy()
    cfg = plan.config()
    assert cfg["waves_per_cu"] in (8, 16, 32) and cfg["msgs_per_lane"] in (1, 2) and cfg["variant"] in (0, 1)
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
def test_full_size_sm3_uneven_sampled(hb):
    """SM3 over 2^22 messages with lengths uniform on 0..4096 (about 8 GiB), bucketed plan
    as timed by the benchmark; 20,000 sampled digests plus the longest and shortest
    messages checked against the oracle one by one."""
    import torch

    b = workloads.cfg_sm3_uneven(device="cuda")
    print(f"case full sm3 uneven n={b.n}", flush=True)
    plan = hb.Plan(b.n, flags=hb.PLAN_GRAPH)
    got = plan.run(b.messages, b.offsets, b.lengths, algo=2)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([rng.choice(b.n, 20_000, replace=False), [0, b.n - 1],
                                    np.argsort(b.lengths)[:50], np.argsort(b.lengths)[-50:]]))
    _check_sampled(hb, b, idx, got, 2)
    plan.close()


@pytest.mark.slow
def test_full_size_mixed_8gib_sampled(hb):
    """Mixed 8 GiB batch (log-normal lengths, median 512 B, cap 1 MiB), one fused
    persistent launch; sampled digests including the 100 longest messages."""
    import torch

    b = workloads.cfg_mixed_8gib(device="cuda")
    print(f"case full mixed n={b.n}", flush=True)
    plan = hb.Plan(b.n, flags=hb.PLAN_GRAPH)
    got = plan.run(b.messages, b.offsets, b.lengths, algos=b.algos)
    torch.cuda.synchronize()
    rng = np.random.default_rng(4)
    idx = np.unique(np.concatenate([rng.choice(b.n, 20_000, replace=False), np.argsort(b.lengths)[-100:]]))
    _check_sampled(hb, b, idx, got, b.algos)
    plan.close()


def _check_sampled(hb, b, idx, got, algo):
    import torch

    lens = b.lengths[idx]
    offs = b.offsets[idx]
    parts = [b.messages[int(o):int(o + L)].cpu().numpy() for o, L in zip(offs, lens)]
    host = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
    noffs = workloads.packed(lens)
    a = algo[idx] if isinstance(algo, np.ndarray) else algo
    want = oracle.hash_batch(a, host, noffs, lens, out_stride=got.shape[1])
    assert_same(got[torch.from_numpy(idx).cuda()].cpu().numpy(), want, "sampled full size")


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
        for var in (0, 1):
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
