"""Helpers shared by the GPU parity tests (no hash arithmetic here)."""
import numpy as np

import oracle

CANARY = 0xA5


def to_dev(a):
    import torch

    if a.dtype == np.uint64:
        a = a.astype(np.int64)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def guarded_out(n, stride, guard=256):
    """A digest buffer with canary bytes before and after the n*stride slots."""
    import torch

    buf = torch.full((guard + n * stride + guard,), CANARY, dtype=torch.uint8, device="cuda")
    return buf, buf[guard:guard + n * stride].view(n, stride)


def check_guard(buf, n, stride, guard=256):
    h = buf.cpu().numpy()
    assert (h[:guard] == CANARY).all(), "write before the digest buffer"
    assert (h[guard + n * stride:] == CANARY).all(), "write past the digest buffer"


def oracle_digests(algo, msgs, offs, lens, stride=None):
    return oracle.hash_batch(algo, msgs, offs, lens, out_stride=stride)


def assert_same(got, want, what=""):
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape, (got.shape, want.shape)
    bad = np.nonzero((got != want).any(axis=1))[0] if got.ndim == 2 else np.nonzero(got != want)[0]
    assert bad.size == 0, f"{what}: {bad.size} mismatching digests, first at {bad[:8].tolist()}"
