"""The allocation-free batched entry point (hash_batch_bucketed_noalloc): its digests equal
hb_plan_run's (and the oracle's) on two calls in a row, the second with a smaller input,
through the C ABI; sizes past its static workspace are rejected before any launch."""
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


def _mixed(seed, total, long_lens):
    """Mixed-algorithm batch with log-normal lengths, a few long messages (direct chains)
    and an empty one."""
    b = workloads.mixed_batch(total, seed=seed, cap=1 << 16)
    rng = np.random.default_rng(seed)
    lens = b.lengths.copy()
    lens[rng.choice(b.n, len(long_lens), replace=False)] = long_lens
    offs = workloads.packed(lens)
    msgs = workloads.host_random_bytes(int(lens.sum()), seed)
    return msgs, offs, lens, b.algos


def test_noalloc_matches_plan_run_twice(hb):
    import torch

    big = _mixed(31, 6_000_000, [1 << 18, 300_000, 70_000, 0, 20_000])
    small = _mixed(32, 400_000, [100_000, 0])
    assert big[2].size > small[2].size
    for k, (msgs, offs, lens, algos) in enumerate((big, small)):
        n = offs.size
        print(f"case noalloc call {k} n={n} bytes={int(lens.sum())}", flush=True)
        buf, out = guarded_out(n, 32)
        hb.hash_batch_bucketed_noalloc(msgs, offs, lens, algos=algos, out=out)
        torch.cuda.synchronize()
        check_guard(buf, n, 32)
        plan = hb.Plan(n)
        ref = plan.run(msgs, offs, lens, algos=algos).cpu().numpy()
        plan.close()
        got = out.cpu().numpy()
        assert_same(got, ref, f"noalloc vs hb_plan_run, call {k}")
        assert_same(got, oracle.hash_batch(algos, msgs, offs, lens), f"noalloc vs oracle, call {k}")


@pytest.mark.parametrize("algo", [0, 1, 2])
def test_noalloc_single_algo_twice(hb, algo):
    for k, (n, cap) in enumerate(((50_000, 5000), (3_000, 300))):
        b = workloads.uniform_lengths_batch(algo, n, cap, seed=40 + k)
        print(f"case noalloc single algo={algo} call {k} n={b.n}", flush=True)
        got = hb.hash_batch_bucketed_noalloc(b.messages, b.offsets, b.lengths, algo=algo).cpu().numpy()
        plan = hb.Plan(b.n)
        ref = plan.run(b.messages, b.offsets, b.lengths, algo=algo).cpu().numpy()
        plan.close()
        assert_same(got, ref, f"noalloc vs hb_plan_run algo={algo} call {k}")
        assert_same(got, oracle.hash_batch(algo, b.messages, b.offsets, b.lengths), "noalloc vs oracle")


def test_noalloc_limits(hb):
    import torch

    n = hb.NOALLOC_MAX_N + 1
    lens = torch.zeros(n, dtype=torch.int64, device="cuda")
    out = torch.empty((n, 16), dtype=torch.uint8, device="cuda")
    msgs = torch.zeros(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(hb.HBError) as ei:
        hb.hash_batch_bucketed_noalloc(msgs, lens, lens, algo=0, out=out)
    assert ei.value.status == hb.HB_EINVAL and "2^20" in str(ei.value)
    # n == 0 is a no-op
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    assert hb.hash_batch_bucketed_noalloc(msgs, e, e, algo=2).shape == (0, 32)
    # exactly the limit: all empty messages
    n = hb.NOALLOC_MAX_N
    got = hb.hash_batch_bucketed_noalloc(msgs, lens[:n], lens[:n], algo=0, out=out[:n]).cpu().numpy()
    want = oracle.hash_batch(0, np.zeros(0, np.uint8), np.zeros(1, np.uint64), np.zeros(1, np.uint64))
    assert (got == want[0]).all()
