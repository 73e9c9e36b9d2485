"""Incremental hashing (init / update / final with device-resident chaining state):
hashing a message in whole-block pieces over several launches gives the digest of the
whole message, bit-exact against the oracle's one-shot digest."""
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


def _split(rng, L, k):
    """k whole-block cut points inside [0, L], then the final piece."""
    nblk = L // 64
    cuts = np.sort(rng.integers(0, nblk + 1, size=k)) * 64
    return [0, *cuts.tolist()]


@pytest.mark.parametrize("algo", [0, 1, 2])
def test_pieces_equal_one_shot(hb, algo):
    rng = np.random.default_rng(algo + 30)
    n = 700
    lens = rng.integers(0, 5000, size=n).astype(np.uint64)
    lens[:8] = [0, 55, 56, 63, 64, 119, 128, 4096]
    offs = workloads.packed(lens)
    msgs = workloads.host_random_bytes(int(lens.sum()), seed=algo + 31)
    k = 4
    cuts = np.array([_split(rng, int(L), k) for L in lens], dtype=np.uint64)  # (n, k+1)
    print(f"case stream algo={algo}", flush=True)
    st = hb.hash_init(algo, n)
    for j in range(k):
        a, b = cuts[:, j], cuts[:, j + 1]
        hb.hash_update(algo, st, msgs, offs + a, b - a)
    out = hb.hash_final(algo, st, msgs, offs + cuts[:, k], lens - cuts[:, k]).cpu().numpy()
    assert_same(out, oracle.hash_batch(algo, msgs, offs, lens), "pieces vs one shot")


@pytest.mark.parametrize("algo", [0, 1, 2])
def test_long_message_across_launches_and_state_export(hb, algo):
    import torch

    L = (4 << 20) + 13
    msg = workloads.host_random_bytes(L, seed=40 + algo)
    st = hb.hash_init(algo, 1)
    piece = 256 << 10
    pos = 0
    while L - pos > piece:
        hb.hash_update(algo, st, msg, np.array([pos], np.uint64), np.array([piece], np.uint64))
        pos += piece
        if pos == 4 * piece:  # suspend: copy the state out and back in
            saved = st.cpu().clone()
            st = torch.zeros_like(st)
            st.copy_(saved.cuda())
    d = hb.hash_final(algo, st, msg, np.array([pos], np.uint64), np.array([L - pos], np.uint64))
    assert d.cpu().numpy()[0].tobytes() == oracle.hash_one(algo, msg)


def test_partial_block_update_marks_state_invalid(hb):
    msg = workloads.host_random_bytes(1000, seed=5)
    st = hb.hash_init(2, 2)
    hb.hash_update(2, st, msg, np.array([0, 0], np.uint64), np.array([64, 63], np.uint64))
    flags = st.cpu().numpy()[:, 5]
    assert flags.tolist() == [0, 1]
    d = hb.hash_final(2, st, msg, np.array([64, 63], np.uint64), np.array([100, 100], np.uint64)).cpu().numpy()
    assert d[0].tobytes() == oracle.hash_one(2, msg[:164])
    assert not d[1].any()
