"""The serving loop in resident mode (HB_SERVER_MODE=resident): one launch of the serving
kernel stays on the device while requests keep coming, and each request's work items join
it as soon as its payload has landed.  Every digest against the oracle; the host ending the
kernel's bounded wait; the kernel leaving on its own when idle and the loop relaunching it."""
import time

import numpy as np
import pytest

from paper_2407_09333_amd import workloads
from tests.gpu_util import assert_same
from tests.test_gpu_host_serving import _long_chain_requests, _requests, _want

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hb():
    import torch

    assert torch.cuda.is_available()
    from paper_2407_09333_amd import hb as _hb

    return _hb


@pytest.fixture
def resident(monkeypatch):
    monkeypatch.setenv("HB_SERVER_MODE", "resident")


def test_resident_results_match_oracle_and_alone(hb, resident):
    reqs = _requests(60, seed=21)
    print("case resident parity", flush=True)
    srv = hb.Server(hbm_budget_bytes=1 << 30, max_slots=32)
    tickets = [srv.submit(r.messages, r.offsets, r.lengths, algo=r.algo, algos=r.algos) for r in reqs]
    outs = [srv.wait(t, timeout_ms=60_000) for t in tickets]
    for r, o in zip(reqs, outs):
        assert_same(o, _want(r), "resident serving")
        if r.algos is None:
            alone = hb.hash_batch(r.algo, r.messages, r.offsets, r.lengths).cpu().numpy()
        else:
            alone = hb.hash_batch_mixed(r.algos, r.messages, r.offsets, r.lengths).cpu().numpy()
        assert_same(o, alone, "alone vs mix")
    assert srv.stats()["completed"] == len(reqs)
    for t in tickets:
        tr = srv.trace(t)
        assert tr["submit"] <= tr["admit"] <= tr["stage_begin"] <= tr["stage_end"] <= tr["launch"] <= tr["done"]
        assert tr["stage_end"] - 1e-3 <= tr["h2d_done"] <= tr["exec_begin"] + 1e-3
        assert tr["exec_begin"] <= tr["exec_end"] <= tr["done"] + 1e-3
    srv.close()


@pytest.mark.parametrize("latency_items", [None, "0", "1000000"])
def test_resident_long_chains(hb, resident, monkeypatch, latency_items):
    """Requests holding long chains, with item formation as configured by default, never
    cooperative (every item one message per lane) and always cooperative (each algorithm's
    two longest classes of >= 128 blocks in items of <= 4 messages run by whole waves)."""
    if latency_items is not None:
        monkeypatch.setenv("HB_SERVER_RESIDENT_LATENCY_ITEMS", latency_items)
    reqs = _long_chain_requests(seed=62)
    print(f"case resident long chains latency_items={latency_items}", flush=True)
    srv = hb.Server(hbm_budget_bytes=1 << 30, max_slots=64)
    tickets = [srv.submit(r.messages, r.offsets, r.lengths, algo=r.algo, algos=r.algos) for r in reqs]
    for r, t in zip(reqs, tickets):
        assert_same(srv.wait(t, timeout_ms=60_000), _want(r), "resident long chains")
    srv.close()


@pytest.mark.slow
def test_resident_benchmark_distribution_burst(hb, resident):
    """600 requests of the serving benchmark's distribution submitted at once."""
    reqs = workloads.serving_requests(600, 1e9, seed=18, mixed_fraction=0.3)
    print(f"case resident burst n_req={len(reqs)}", flush=True)
    srv = hb.Server(hbm_budget_bytes=4 << 30, max_slots=256)
    tickets = [srv.submit(r.messages, r.offsets, r.lengths, algo=r.algo, algos=r.algos) for r in reqs]
    for r, t in zip(reqs, tickets):
        assert_same(srv.wait(t, timeout_ms=120_000), _want(r), "resident burst")
    assert srv.stats()["completed"] == len(reqs)
    srv.close()


def test_resident_budget_and_cancel(hb, resident):
    rng = np.random.default_rng(72)
    reqs = []
    for r in range(24):
        lens = rng.integers(2000, 6000, size=200).astype(np.uint64)
        reqs.append(workloads.Request(0.0, r % 3, None, lens, workloads.host_random_bytes(int(lens.sum()), 600 + r),
                                      workloads.packed(lens)))
    print("case resident budget/cancel", flush=True)
    srv = hb.Server(hbm_budget_bytes=2 << 20, max_slots=2)
    tickets = [srv.submit(r.messages, r.offsets, r.lengths, algo=r.algo) for r in reqs]
    cancelled = {t for t in tickets[8::2] if srv.cancel(t)}
    for r, t in zip(reqs, tickets):
        if t in cancelled:
            with pytest.raises(hb.HBError) as e:
                srv.wait(t, timeout_ms=60_000)
            assert e.value.status == hb.HB_ECANCELED
        else:
            assert_same(srv.wait(t, timeout_ms=60_000), _want(r), "resident after cancels")
    st = srv.stats()
    assert st["peak_bytes"] <= 2 << 20 and st["stalls"] > 0
    srv.close()


def test_resident_idle_exit_and_relaunch(hb, resident):
    """The kernel leaves on its own after a few idle milliseconds; a request arriving later
    starts a new launch, which takes it from where the ring stands."""
    reqs = _requests(6, seed=23)
    print("case resident idle exit and relaunch", flush=True)
    srv = hb.Server(hbm_budget_bytes=256 << 20, max_slots=8)
    for k, r in enumerate(reqs):
        t = srv.submit(r.messages, r.offsets, r.lengths, algo=r.algo, algos=r.algos)
        assert_same(srv.wait(t, timeout_ms=60_000), _want(r), f"resident request {k}")
        time.sleep(0.05)  # well past the 5 ms idle limit
    assert srv.stats()["steps"] >= len(reqs)  # a launch per request: each idled out before the next
    srv.close()


def test_resident_host_ends_the_wait(hb, resident, monkeypatch):
    """Closing the server while the kernel waits for items: with a 20 s idle limit the
    kernel would wait that long on its own; the host's stop flag ends its wait, and close
    returns promptly with every request done."""
    monkeypatch.setenv("HB_SERVER_RESIDENT_IDLE_MS", "20000")
    reqs = _requests(4, seed=24)
    print("case resident host stop", flush=True)
    srv = hb.Server(hbm_budget_bytes=256 << 20, max_slots=8)
    tickets = [srv.submit(r.messages, r.offsets, r.lengths, algo=r.algo, algos=r.algos) for r in reqs]
    for r, t in zip(reqs, tickets):
        assert_same(srv.wait(t, timeout_ms=60_000), _want(r), "resident before stop")
    t0 = time.perf_counter()
    srv.close()  # the kernel is still inside its idle window: the stop flag ends it
    assert time.perf_counter() - t0 < 2.0


@pytest.mark.parametrize("mode", ["steps", "resident"])
def test_collect_traces_and_releases(hb, monkeypatch, mode):
    """Server.collect (wait, trace into an array, release): the trace it writes is the one
    hb_server_trace reports, ordered in time; the record is gone afterwards; a cancelled
    request's status is raised after its record is released."""
    monkeypatch.setenv("HB_SERVER_MODE", mode)
    reqs = _requests(12, seed=33)
    print(f"case collect {mode}", flush=True)
    srv = hb.Server(hbm_budget_bytes=1 << 30, max_slots=16)
    tickets = [srv.submit(r.messages, r.offsets, r.lengths, algo=r.algo, algos=r.algos) for r in reqs]
    rows = np.zeros((len(tickets), len(srv.TRACE_NAMES)))
    for k, t in enumerate(tickets):
        srv.collect(t, rows[k])
        tm = dict(zip(srv.TRACE_NAMES, rows[k]))
        assert tm["submit"] <= tm["admit"] <= tm["stage_begin"] <= tm["stage_end"] <= tm["done"]
        assert tm["exec_begin"] <= tm["exec_end"] <= tm["done"] + 1e-3
        with pytest.raises(hb.HBError):
            srv.trace(t)  # released
    assert srv.stats()["completed"] == len(reqs)
    srv.close()
    # requests queued behind a tiny budget, some cancelled before admission: collect raises
    # HB_ECANCELED for those, and every record is released either way
    rng = np.random.default_rng(34)
    lens = [rng.integers(2000, 6000, size=200).astype(np.uint64) for _ in range(12)]
    srv = hb.Server(hbm_budget_bytes=2 << 20, max_slots=2)
    tickets = [srv.submit(workloads.host_random_bytes(int(L.sum()), 700 + k), workloads.packed(L), L, algo=k % 3)
               for k, L in enumerate(lens)]
    cancelled = {t for t in tickets[6::2] if srv.cancel(t)}
    row = np.zeros(len(srv.TRACE_NAMES))
    for t in tickets:
        if t in cancelled:
            with pytest.raises(hb.HBError) as e:
                srv.collect(t, row)
            assert e.value.status == hb.HB_ECANCELED
        else:
            srv.collect(t, row)
        with pytest.raises(hb.HBError):
            srv.trace(t)
    assert cancelled
    srv.close()
