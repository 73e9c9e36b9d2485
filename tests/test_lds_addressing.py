"""Host model of the LDS-staged plain kernel's addressing (k_plain_lds in hb_kernels.hip),
checked on the CPU for the lengths the kernel takes.  The index arithmetic below is the
kernel's, restated: lane (q, p) = (lane / 8, lane % 8) of load j of burst k reads 16 bytes
at k 128 + 8 j len + q len + (p ^ q) 16 from the wave's base and writes them to slot
64 j + lane of the wave's LDS slice; lane L reads chunk c of its message back from slot
8 L + (c ^ (L % 8)).  Properties: every load stays inside the buffer resource's range (the
wave's 64 messages, 64 len bytes); each load instruction reads 128 whole bytes of each of
eight messages; a wave's loads read its messages' first 128 nburst bytes exactly once; the
read-back gives each lane its own message's bytes in order; and the eight lanes reading
one chunk position hit eight different 16-byte bank groups."""
import numpy as np
import pytest

LENS = [128, 132, 256, 384, 512, 640, 768, 896, 1024, 1028, 1152, 2048, 4096, 65536, (1 << 25) - 4]


def loads(length, bursts=None):
    """(k, j, start offsets of the 64 lanes) for every load instruction of a whole wave
    (or of the bursts listed)."""
    nfast = length // 64
    nburst = nfast // 2
    lane = np.arange(64, dtype=np.int64)
    q, p = lane // 8, lane % 8
    voff = q * length + (p ^ q) * 16
    for k in (range(nburst) if bursts is None else bursts):
        for j in range(8):
            yield k, j, k * 128 + 8 * j * length + voff


@pytest.mark.parametrize("length", LENS)
def test_loads_stay_in_range_and_cover_each_prefix_once(length):
    nburst = (length // 64) // 2
    rng_end = 64 * length
    assert rng_end < 1 << 31  # the resource's 32-bit range
    if length > 4096:  # the byte map would be large: the first and the furthest bursts
        for k, j, start in loads(length, bursts=(0, nburst - 1)):
            assert start.min() >= 0 and (start + 16).max() <= rng_end
        return
    seen = np.zeros(rng_end, dtype=np.int32)
    for k, j, start in loads(length):
        assert start.min() >= 0 and (start + 16).max() <= rng_end
        np.add.at(seen, (start[:, None] + np.arange(16)).ravel(), 1)
        # one instruction: 128 whole bytes of each of messages 8j .. 8j + 7
        msgs = (start // length)
        assert sorted(set(msgs.tolist())) == list(range(8 * j, 8 * j + 8))
        for m in range(8 * j, 8 * j + 8):
            got = np.sort(start[msgs == m] - m * length)
            assert got.tolist() == [k * 128 + 16 * c for c in range(8)]
    per_msg = seen.reshape(64, length)
    assert (per_msg[:, :128 * nburst] == 1).all()
    assert (per_msg[:, 128 * nburst:] == 0).all()


def test_read_back_is_each_lanes_own_message_in_order():
    lane = np.arange(64)
    q, p = lane // 8, lane % 8
    for j in range(8):
        # slot 64 j + lane holds chunk (p ^ q) of message 8 j + q
        slot_msg = {64 * j + int(l): (8 * j + int(qq), int(pp ^ qq)) for l, qq, pp in zip(lane, q, p)}
        for L in range(8 * j, 8 * j + 8):
            sw = L % 8
            for c in range(8):
                assert slot_msg[8 * L + (c ^ sw)] == (L, c)


def test_read_back_bank_groups_differ():
    # eight consecutive lanes read the same chunk position c: their 16-byte slots fall in
    # eight different groups of four 4-byte banks (16 groups in a 64-bank LDS row)
    for c in range(8):
        for base in range(0, 64, 8):
            groups = {(8 * L + (c ^ (L % 8))) % 16 for L in range(base, base + 8)}
            assert len(groups) == 8
