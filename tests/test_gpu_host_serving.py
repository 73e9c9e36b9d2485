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


@pytest.fixture
def zero_copy_limit():
    """Set HB_HOST_ZERO_COPY_MAX for one test (read by the library at each call)."""
    import os

    old = os.environ.get("HB_HOST_ZERO_COPY_MAX")

    def set_limit(v):
        os.environ["HB_HOST_ZERO_COPY_MAX"] = str(v)

    yield set_limit
    if old is None:
        os.environ.pop("HB_HOST_ZERO_COPY_MAX", None)
    else:
        os.environ["HB_HOST_ZERO_COPY_MAX"] = old


@pytest.mark.parametrize("chunk", [1 << 16, 1 << 20, 64 << 20])
def test_host_pipeline_mixed(hb, zero_copy_limit, chunk):
    zero_copy_limit(0)  # the chunked copy-engine path, whatever the batch size
    b = workloads.mixed_batch(3_000_000, seed=21, cap=1 << 17)
    print(f"case host pipeline chunk={chunk} n={b.n}", flush=True)
    got = hb.hash_batch_host(b.messages, b.offsets, b.lengths, algos=b.algos, chunk_bytes=chunk)
    assert_same(got, oracle.hash_batch(b.algos, b.messages, b.offsets, b.lengths), "host mixed")


def test_host_default_path_mixed(hb):
    """A 3 MB mixed batch at the default limit (hashed in place from pinned memory)."""
    b = workloads.mixed_batch(3_000_000, seed=22, cap=1 << 17)
    print(f"case host default path n={b.n}", flush=True)
    got = hb.hash_batch_host(b.messages, b.offsets, b.lengths, algos=b.algos)
    assert_same(got, oracle.hash_batch(b.algos, b.messages, b.offsets, b.lengths), "host default")


@pytest.mark.parametrize("frac", [0.0, 0.1, 0.5, 1.0])
def test_host_cpu_gpu_split(hb, zero_copy_limit, frac):
    """The CPU + GPU split: host cores take the trailing messages holding about `frac` of
    the payload, the GPU path the rest (through the copy engine here, as for a large
    batch); the merged digests equal the oracle's."""
    zero_copy_limit(0)
    b = workloads.mixed_batch(4_000_000, seed=23, cap=1 << 17)
    al = b.algos.copy()
    al[::53] = 11
    print(f"case host split frac={frac} n={b.n}", flush=True)
    got = hb.hash_batch_host_split(b.messages, b.offsets, b.lengths, algos=al, cpu_fraction=frac, cpu_threads=4)
    valid = al < 3
    want = np.zeros((b.n, 32), np.uint8)
    want[valid] = oracle.hash_batch(al[valid], b.messages, b.offsets[valid], b.lengths[valid])
    assert_same(got, want, f"split {frac}")
    single = hb.hash_batch_host_split(b.messages, b.offsets, b.lengths, algo=2, cpu_fraction=frac)
    assert_same(single, oracle.hash_batch(2, b.messages, b.offsets, b.lengths), f"split sm3 {frac}")


def test_host_cpu_gpu_split_rejects_bad_fraction(hb):
    z = np.zeros(1, np.uint64)
    with pytest.raises(hb.HBError) as e:
        hb.hash_batch_host_split(np.zeros(1, np.uint8), z, z, algo=0, cpu_fraction=1.5)
    assert e.value.status == hb.HB_EINVAL


def test_host_pipeline_single_algo_overlapping(hb):
    data = workloads.host_random_bytes(200_000, seed=5)
    rng = np.random.default_rng(5)
    offs = rng.integers(0, 100_000, size=3000).astype(np.uint64)
    lens = rng.integers(0, 100_000, size=3000).astype(np.uint64)
    print("case host overlapping", flush=True)
    got = hb.hash_batch_host(data, offs, lens, algo=1, chunk_bytes=4 << 20)
    assert_same(got, oracle.hash_batch(1, data, offs, lens), "host overlapping")


@pytest.mark.parametrize("limit", [1 << 40, 0])
def test_host_small_batches_zero_copy_and_copy_engine(hb, zero_copy_limit, limit):
    """Small batches hashed in place from pinned memory (limit 2^40) and through the copy
    engine (limit 0) give the oracle's digests."""
    zero_copy_limit(limit)
    # 4,096 x 55 B MD5, one block each
    data = workloads.host_random_bytes(4096 * 55, seed=1)
    offs = np.arange(4096, dtype=np.uint64) * np.uint64(55)
    lens = np.full(4096, 55, np.uint64)
    print(f"case host small limit={limit} md5 4096x55", flush=True)
    assert_same(hb.hash_batch_host(data, offs, lens, algo=0), oracle.hash_batch(0, data, offs, lens), "md5 55")
    # every length 0..300 at odd offsets, each algorithm, then mixed with unknown ids
    rng = np.random.default_rng(31)
    lens = np.arange(301, dtype=np.uint64)
    offs = (np.cumsum(lens) - lens + rng.integers(0, 7, size=lens.size).cumsum()).astype(np.uint64)
    data = workloads.host_random_bytes(int(offs[-1] + lens[-1]) + 8, seed=32)
    for a in range(3):
        print(f"case host small limit={limit} algo={a} lengths 0..300", flush=True)
        assert_same(hb.hash_batch_host(data, offs, lens, algo=a), oracle.hash_batch(a, data, offs, lens), "lengths")
    ids = rng.integers(0, 3, size=lens.size).astype(np.uint8)
    ids[::17] = 7
    print(f"case host small limit={limit} mixed", flush=True)
    valid = ids < 3
    want = np.zeros((lens.size, 32), np.uint8)  # an unknown id gives an all-zero slot
    want[valid] = oracle.hash_batch(ids[valid], data, offs[valid], lens[valid])
    assert_same(hb.hash_batch_host(data, offs, lens, algos=ids), want, "mixed small")
    # overlapping messages, and one empty batch of many empty messages
    offs = rng.integers(0, 1000, size=500).astype(np.uint64)
    lens = rng.integers(0, 1000, size=500).astype(np.uint64)
    print(f"case host small limit={limit} overlapping", flush=True)
    assert_same(hb.hash_batch_host(data, offs, lens, algo=2), oracle.hash_batch(2, data, offs, lens), "overlap")
    z = np.zeros(3000, np.uint64)
    assert_same(hb.hash_batch_host(data, z, z, algo=1), oracle.hash_batch(1, data, z, z), "empties")


def test_host_zero_copy_limit_boundary(hb, zero_copy_limit):
    """Batches just under and just over the zero-copy limit agree with each other and the
    oracle (the two paths meet at the limit)."""
    zero_copy_limit(64 * 1024)
    data = workloads.host_random_bytes(64 * 1024 + 64, seed=33)
    for n_bytes in (64 * 1024, 64 * 1024 + 64):
        n = n_bytes // 64
        offs = np.arange(n, dtype=np.uint64) * np.uint64(64)
        lens = np.full(n, 64, np.uint64)
        print(f"case host zero-copy boundary bytes={n_bytes}", flush=True)
        assert_same(hb.hash_batch_host(data, offs, lens, algo=1), oracle.hash_batch(1, data, offs, lens), "boundary")


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


@pytest.mark.slow
def test_serving_benchmark_distribution_burst(hb):
    """600 requests of the serving benchmark's own distribution (1..10,000 messages each,
    log-normal lengths capped at 64 KiB, a third mixing algorithms per message), submitted
    at once -- staging groups, both request classes, both compute streams and the kernel
    copies all in play; every digest against the oracle."""
    reqs = workloads.serving_requests(600, 1e9, seed=17, mixed_fraction=0.3)
    print(f"case serving burst n_req={len(reqs)} msgs={sum(r.lengths.size for r in reqs)}", flush=True)
    srv = hb.Server(hbm_budget_bytes=4 << 30, max_slots=256)
    tickets = [srv.submit(r.messages, r.offsets, r.lengths, algo=r.algo, algos=r.algos) for r in reqs]
    outs = [srv.wait(t, timeout_ms=120_000) for t in tickets]
    for r, o in zip(reqs, outs):
        assert_same(o, _want(r), "serving burst")
    assert srv.stats()["completed"] == len(reqs)
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


def _long_chain_requests(seed=61):
    """Requests around the long-chain thresholds: short ones, and ones holding messages of
    255 / 256 blocks (L = 16,311 / 16,312), 64 KiB and 200,000 bytes, single-algorithm and
    mixed."""
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(14):
        cnt = int(rng.integers(1, 400))
        lens = rng.integers(0, 3000, size=cnt).astype(np.uint64)
        if r % 2:
            k = min(cnt, 4)
            lens[rng.choice(cnt, k, replace=False)] = [16_311, 16_312, 65_536, 200_000][:k]
        offs = workloads.packed(lens)
        msgs = workloads.host_random_bytes(int(lens.sum()), seed * 1000 + r)
        algos = rng.integers(0, 3, size=cnt).astype(np.uint8) if r % 3 == 0 else None
        reqs.append(workloads.Request(0.0, None if algos is not None else r % 3, algos, lens, msgs, offs))
    return reqs


@pytest.mark.parametrize("env", [{}, {"HB_SERVER_LONG_PLAN_FLAGS": "8"}, {"HB_SERVER_LONG_PLAN_FLAGS": "0"},
                                 {"HB_SERVER_LONG_STREAMS": "2", "HB_SERVER_LONG_PLAN_FLAGS": "16"},
                                 {"HB_SERVER_LONG_PLAN_FLAGS": "16", "HB_LONG_MIN_BLOCKS": "2",
                                  "HB_LONG_SCRATCH_MB": "1"},
                                 {"HB_SERVER_COPY": "kernel"}, {"HB_SERVER_COPY_STREAMS": "2"},
                                 {"HB_SERVER_STAGERS": "1"},
                                 {"HB_SERVER_STAGERS": "8", "HB_SERVER_COPY_STREAMS": "2", "HB_SERVER_LONG_STREAMS": "2"}],
                         ids=["default_one_launch", "no_long_path", "long_path_side_stream", "two_long_streams",
                              "direct_chains", "kernel_copies", "two_copy_streams", "one_stager",
                              "eight_stagers_two_copy_two_long"])
def test_serving_long_chain_steps(hb, monkeypatch, env):
    """Requests holding long chains go to long-chain steps, whose plans by default run the
    longest chains rounds-only from precomputed schedule words (or, with a scratch too
    small for them, as direct chains) in the same launch as the bulk; also with the chains
    on a side stream, or without the long-chain path; with one or two long-chain streams;
    payload copied by the copy engine (on one or two copy streams) or by kernels.  Every
    digest against the oracle."""
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    reqs = _long_chain_requests()
    print(f"case serving long chains env={env}", flush=True)
    srv = hb.Server(hbm_budget_bytes=1 << 30, max_slots=64)
    tickets = [srv.submit(r.messages, r.offsets, r.lengths, algo=r.algo, algos=r.algos) for r in reqs]
    outs = [srv.wait(t, timeout_ms=60_000) for t in tickets]
    for r, o in zip(reqs, outs):
        assert_same(o, _want(r), "serving long chains")
    assert srv.stats()["completed"] == len(reqs)
    srv.close()


def test_serving_cancel_and_release(hb):
    """Requests held back by a small budget can be cancelled while queued: they finish with
    HB_ECANCELED and their slots untouched; the rest complete bit-exact.  Admitted or
    finished requests cannot be cancelled; finished ones can be released."""
    rng = np.random.default_rng(71)
    reqs = []
    for r in range(30):
        lens = rng.integers(2000, 6000, size=200).astype(np.uint64)  # ~0.8 MB each
        offs = workloads.packed(lens)
        reqs.append(workloads.Request(0.0, r % 3, None, lens, workloads.host_random_bytes(int(lens.sum()), 500 + r),
                                      offs))
    print("case serving cancel/release", flush=True)
    srv = hb.Server(hbm_budget_bytes=2 << 20, max_slots=2)
    tickets = [srv.submit(r.messages, r.offsets, r.lengths, algo=r.algo) for r in reqs]
    cancelled = {t for t in tickets[10::2] if srv.cancel(t)}
    assert len(cancelled) >= 5  # the budget holds all but a few requests back
    for r, t in zip(reqs, tickets):
        if t in cancelled:
            with pytest.raises(hb.HBError) as e:
                srv.wait(t, timeout_ms=60_000)
            assert e.value.status == hb.HB_ECANCELED
        else:
            assert_same(srv.wait(t, timeout_ms=60_000), _want(r), "serving after cancels")
    assert srv.cancel(tickets[0]) is False  # finished: nothing to cancel
    assert srv.stats()["completed"] == len(reqs) - len(cancelled)
    for t in tickets:
        srv.release(t)
    with pytest.raises(hb.HBError) as e:
        srv.release(tickets[0])
    assert e.value.status == hb.HB_EINVAL
    srv.close()
