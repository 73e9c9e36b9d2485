"""Host-resident inputs (chunked H2D overlapped with hashing) and the serving loop:
bit-exact against the oracle, alone equals in the mix, budget admission."""
import threading
import time

import numpy as np
import pytest

import oracle
from paper_2407_09333_amd import workloads
from tests.gpu_util import assert_same

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hb():
    import torch

    assert torch.cuda.is_available()
    from paper_2407_09333_amd import hb as _hb

    return _hb


@pytest.mark.parametrize("chunk", [1 << 16, 1 << 20, 64 << 20])
def test_host_pipeline_mixed(hb, chunk):
    b = workloads.mixed_batch(3_000_000, seed=21, cap=1 << 17)
    print(f"case host pipeline chunk={chunk} n={b.n}", flush=True)
    got = hb.hash_batch_host(b.messages, b.offsets, b.lengths, algos=b.algos, chunk_bytes=chunk)
    assert_same(got, oracle.hash_batch(b.algos, b.messages, b.offsets, b.lengths), "host mixed")


def test_host_pipeline_single_algo_overlapping(hb):
    data = workloads.host_random_bytes(200_000, seed=5)
    rng = np.random.default_rng(5)
    offs = rng.integers(0, 100_000, size=3000).astype(np.uint64)
    lens = rng.integers(0, 100_000, size=3000).astype(np.uint64)
    print("case host overlapping", flush=True)
    got = hb.hash_batch_host(data, offs, lens, algo=1, chunk_bytes=4 << 20)
    assert_same(got, oracle.hash_batch(1, data, offs, lens), "host overlapping")


def _requests(k, seed=5, rate=1e9, mixed_fraction=0.3):
    return workloads.serving_requests(k, rate, seed=seed, max_count=2000, mixed_fraction=mixed_fraction)


def _want(r):
    a = r.algos if r.algos is not None else r.algo
    return oracle.hash_batch(a, r.messages, r.offsets, r.lengths)


def test_serving_results_match_oracle_and_alone(hb):
    reqs = _requests(60)
    print("case serving parity", flush=True)
    srv = hb.Server(hbm_budget_bytes=1 << 30, max_slots=32)
    tickets = [srv.submit(r.messages, r.offsets, r.lengths, algo=r.algo, algos=r.algos) for r in reqs]
    outs = [srv.wait(t, timeout_ms=60_000) for t in tickets]
    for r, o in zip(reqs, outs):
        assert_same(o, _want(r), "serving")
        # alone: the same request through the plain kernel
        if r.algos is None:
            alone = hb.hash_batch(r.algo, r.messages, r.offsets, r.lengths).cpu().numpy()
        else:
            alone = hb.hash_batch_mixed(r.algos, r.messages, r.offsets, r.lengths).cpu().numpy()
        assert_same(o, alone, "alone vs mix")
    st = srv.stats()
    assert st["completed"] == len(reqs)
    for t in tickets:
        tm = srv.times(t)
        assert tm["submit"] <= tm["admit"] <= tm["done"]
        tr = srv.trace(t)
        assert tr["submit"] == tm["submit"] and tr["done"] == tm["done"] and tr["h2d_done"] == tm["h2d_done"]
        # host-clock stamps in order; device-clock stamps in order; the two clocks agree to 1 ms
        assert tr["submit"] <= tr["admit"] <= tr["stage_begin"] <= tr["stage_end"] <= tr["launch"] <= tr["done"]
        assert tr["exec_begin"] <= tr["exec_end"]
        assert tr["stage_end"] - 1e-3 <= tr["h2d_done"] <= tr["exec_begin"] + 1e-3
        assert tr["launch"] - 1e-3 <= tr["exec_begin"] and tr["exec_end"] <= tr["done"] + 1e-3
    srv.close()


def test_serving_budget_admission_never_overcommits(hb):
    reqs = _requests(40, seed=8, mixed_fraction=0.0)
    biggest = max(int(r.lengths.sum()) for r in reqs)
    budget = ((biggest + 255) // 256) * 256 * 2
    print(f"case serving budget={budget}", flush=True)
    srv = hb.Server(hbm_budget_bytes=budget, max_slots=8)
    tickets = [srv.submit(r.messages, r.offsets, r.lengths, algo=r.algo) for r in reqs]
    for r, t in zip(reqs, tickets):
        assert_same(srv.wait(t, timeout_ms=60_000), _want(r), "budgeted")
    st = srv.stats()
    assert st["peak_bytes"] <= budget
    assert st["stalls"] > 0
    srv.close()


def test_serving_rejects_alone(hb):
    srv = hb.Server(hbm_budget_bytes=1 << 20, max_slots=4)
    good = _requests(3, seed=9, mixed_fraction=0.0)
    big = np.zeros(2 << 20, np.uint8)
    with pytest.raises(hb.HBError) as e:
        srv.submit(big, np.zeros(1, np.uint64), np.array([2 << 20], np.uint64), algo=0)
    assert e.value.status == hb.HB_EBUDGET
    with pytest.raises(hb.HBError) as e:
        srv.submit(big, np.zeros(1, np.uint64), np.array([10], np.uint64), algo=5)
    assert e.value.status == hb.HB_EINVAL
    for r in good:
        if r.lengths.sum() < (1 << 20):
            t = srv.submit(r.messages, r.offsets, r.lengths, algo=r.algo)
            assert_same(srv.wait(t, timeout_ms=60_000), _want(r), "after rejects")
    srv.close()


def test_serving_concurrent_submitters(hb):
    reqs = _requests(48, seed=11)
    srv = hb.Server(hbm_budget_bytes=256 << 20, max_slots=16)
    results = {}

    def worker(lo, hi):
        for i in range(lo, hi):
            r = reqs[i]
            t = srv.submit(r.messages, r.offsets, r.lengths, algo=r.algo, algos=r.algos)
            results[i] = srv.wait(t, timeout_ms=60_000)

    print("case serving threads", flush=True)
    th = [threading.Thread(target=worker, args=(k * 12, k * 12 + 12)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for i, r in enumerate(reqs):
        assert_same(results[i], _want(r), "concurrent")
    srv.close()
