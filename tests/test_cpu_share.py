"""The host-core share of a CPU + GPU split (hb_cpu_hash_batch): host code of the library,
independent of the oracle, checked against it bit for bit.  Runs without a GPU."""
import numpy as np
import pytest

import oracle
from paper_2407_09333_amd import workloads


@pytest.fixture(scope="module")
def hb():
    from paper_2407_09333_amd import hb as _hb

    _hb.lib()  # the library loads without a GPU; the host share touches none
    return _hb


@pytest.mark.parametrize("threads", [1, 4])
@pytest.mark.parametrize("algo", [0, 1, 2])
def test_every_length_0_to_300(hb, algo, threads):
    lens = np.arange(301, dtype=np.uint64)
    offs = workloads.packed(lens)
    msgs = workloads.host_random_bytes(int(lens.sum()), seed=61)
    got = hb.cpu_hash_batch(msgs, offs, lens, algo=algo, threads=threads)
    assert np.array_equal(got, oracle.hash_batch(algo, msgs, offs, lens))


def test_mixed_overlapping_unknown_ids_and_long(hb):
    rng = np.random.default_rng(62)
    data = workloads.host_random_bytes(3 << 20, seed=63)
    n = 2000
    offs = rng.integers(0, 1 << 20, size=n).astype(np.uint64)
    lens = rng.integers(0, 5000, size=n).astype(np.uint64)
    lens[:3] = [1 << 20, (1 << 20) + 1, 2 << 20]  # long messages (the FIPS long-message style)
    offs[:3] = 0
    ids = rng.integers(0, 3, size=n).astype(np.uint8)
    ids[::37] = 9
    got = hb.cpu_hash_batch(data, offs, lens, algos=ids, threads=3)
    valid = ids < 3
    want = np.zeros((n, 32), np.uint8)  # an unknown id gives an all-zero slot
    want[valid] = oracle.hash_batch(ids[valid], data, offs[valid], lens[valid])
    assert np.array_equal(got, want)


def test_rejects_bad_arguments(hb):
    z = np.zeros(1, np.uint64)
    with pytest.raises(hb.HBError) as e:
        hb.cpu_hash_batch(np.zeros(1, np.uint8), z, z, algo=7)
    assert e.value.status == hb.HB_EINVAL
