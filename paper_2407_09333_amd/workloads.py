"""Seeded synthetic inputs for batch hashing.

This module only draws random numbers and lays out buffers; it holds none of the hash
arithmetic.  The same arrays feed both the HIP path and the CPU oracle.

Recipes (the paper's own workload -- Sec. V-A.2 -- is itself synthetic: every 9-digit
decimal string; the configurations below are larger synthetic stand-ins):

* message bytes: uniform random.  On the host they are the little-endian bytes of
  ``numpy.random.PCG64(seed).random_raw()`` words (stable across numpy versions); on the
  GPU (multi-GiB buffers) they come from torch's seeded device generator.
* lengths, algorithm ids, request sizes and arrival gaps: ``numpy.random.Generator(
  PCG64(seed + 100))``.
* packing: messages are stored back to back (``offsets[i] = sum of lengths[:i]``), so
  offsets have any byte alignment.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

MD5, SHA1, SM3 = 0, 1, 2


@dataclass
class Batch:
    """A batch of messages in one packed byte buffer.

    ``messages`` is a 1-D uint8 numpy array or torch tensor; ``offsets``/``lengths`` are
    uint64 numpy arrays; ``algos`` is a uint8 array of per-message algorithm ids or None
    when the whole batch uses ``algo``."""

    messages: object
    offsets: np.ndarray
    lengths: np.ndarray
    algo: int | None = None
    algos: np.ndarray | None = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.offsets.size)

    @property
    def total_bytes(self) -> int:
        return int(self.lengths.sum())


def host_random_bytes(nbytes: int, seed: int) -> np.ndarray:
    """nbytes uniform random bytes: LE bytes of PCG64(seed).random_raw() words."""
    words = (nbytes + 7) // 8
    raw = np.random.PCG64(seed).random_raw(max(words, 1)).astype("<u8", copy=False)
    return raw.view(np.uint8)[:nbytes].copy() if nbytes else np.zeros(0, np.uint8)


def device_random_bytes(nbytes: int, seed: int, device="cuda"):
    """nbytes uniform random bytes drawn on the GPU from torch's seeded generator."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return torch.randint(0, 256, (max(nbytes, 1),), dtype=torch.uint8, device=device,
                         generator=g)[:nbytes]


def _random_bytes(nbytes: int, seed: int, device: str):
    if device == "cpu":
        return host_random_bytes(nbytes, seed)
    return device_random_bytes(nbytes, seed, device)


def packed(lengths: np.ndarray) -> np.ndarray:
    """Tight packing: offsets[i] = lengths[0] + ... + lengths[i-1]."""
    lengths = np.asarray(lengths, dtype=np.uint64)
    offs = np.zeros(lengths.size, np.uint64)
    if lengths.size > 1:
        np.cumsum(lengths[:-1], out=offs[1:])
    return offs


def fixed_batch(algo: int, n: int, msg_len: int, seed: int, device: str = "cpu",
                name: str = "") -> Batch:
    """n messages of exactly msg_len bytes, contiguous."""
    msgs = _random_bytes(n * msg_len, seed, device)
    offs = np.arange(n, dtype=np.uint64) * np.uint64(msg_len)
    lens = np.full(n, msg_len, np.uint64)
    return Batch(msgs, offs, lens, algo=algo, name=name, meta={"msg_len": msg_len})


def uniform_lengths_batch(algo: int, n: int, max_len: int, seed: int, device: str = "cpu",
                          min_len: int = 0, name: str = "") -> Batch:
    """n messages with lengths uniform on {min_len..max_len}, tightly packed."""
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    lens = rng.integers(min_len, max_len + 1, size=n, dtype=np.uint64)
    offs = packed(lens)
    msgs = _random_bytes(int(lens.sum()), seed, device)
    return Batch(msgs, offs, lens, algo=algo, name=name)


def lognormal_lengths(rng: np.random.Generator, n: int, median: float, sigma: float,
                      cap: int) -> np.ndarray:
    """floor(exp(N(ln median, sigma^2))) capped at cap."""
    x = np.floor(np.exp(rng.normal(np.log(median), sigma, size=n)))
    return np.minimum(x, cap).astype(np.uint64)


def mixed_batch(total_bytes: int, seed: int, device: str = "cpu", median: float = 512.0,
                sigma: float = 1.5, cap: int = 1 << 20, name: str = "") -> Batch:
    """Algorithm uniform over {MD5, SHA-1, SM3}; log-normal lengths; messages are drawn
    until the next one would push the payload past total_bytes."""
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    chunks = []
    acc = 0
    est = max(16, int(total_bytes / (median * np.exp(sigma * sigma / 2)) * 1.1) + 16)
    while True:
        lens = lognormal_lengths(rng, est, median, sigma, cap)
        cs = np.cumsum(lens, dtype=np.uint64) + np.uint64(acc)
        k = int(np.searchsorted(cs, np.uint64(total_bytes), side="right"))
        chunks.append(lens[:k])
        if k < lens.size:
            break
        acc = int(cs[-1])
        est = max(16, est // 4)
    lens = np.concatenate(chunks)
    algos = rng.integers(0, 3, size=lens.size, dtype=np.uint8)
    offs = packed(lens)
    msgs = _random_bytes(int(lens.sum()), seed, device)
    return Batch(msgs, offs, lens, algos=algos, name=name)


def digits9_batch(n: int, start: int = 0) -> Batch:
    """The paper's workload shape (Sec. V-A.2): messages are 9-character strings over
    '0'..'9' -- here message i is the zero-padded decimal text of start + i."""
    idx = np.arange(start, start + n, dtype=np.int64)
    digits = np.zeros((n, 9), np.uint8)
    v = idx.copy()
    for k in range(8, -1, -1):
        digits[:, k] = (v % 10).astype(np.uint8) + ord("0")
        v //= 10
    msgs = digits.reshape(-1)
    offs = np.arange(n, dtype=np.uint64) * np.uint64(9)
    lens = np.full(n, 9, np.uint64)
    return Batch(msgs, offs, lens, name="digits9")


# --------------------------------------------------------------------------------------
# The benchmark configurations (sizes as stated for each; seeds fixed)
# --------------------------------------------------------------------------------------

def cfg_md5_4096x55(device: str = "cpu") -> Batch:
    """MD5 over 4,096 messages of exactly 55 bytes (one padded block each), seed 1."""
    return fixed_batch(MD5, 4096, 55, seed=1, device=device, name="md5_4096x55")


def cfg_fixed_1m_x_1024(algo: int, device: str = "cpu", n: int = 1 << 20) -> Batch:
    """2^20 messages of 1,024 bytes (16 blocks + a padding block), contiguous, seed 2.
    The same buffer is used for all three algorithms."""
    return fixed_batch(algo, n, 1024, seed=2, device=device, name=f"fixed_{n}x1024")


def cfg_sm3_uneven(device: str = "cpu", n: int = 1 << 22) -> Batch:
    """SM3 over 2^22 messages with lengths uniform on {0..4096}, tightly packed, seed 3."""
    return uniform_lengths_batch(SM3, n, 4096, seed=3, device=device, name=f"sm3_uneven_{n}")


def cfg_mixed_8gib(device: str = "cpu", total_bytes: int = 1 << 33) -> Batch:
    """8 GiB payload, algorithm uniform, log-normal lengths (median 512 B, sigma 1.5, cap
    1 MiB), seed 4."""
    return mixed_batch(total_bytes, seed=4, device=device, name=f"mixed_{total_bytes}")


@dataclass
class Request:
    arrival_s: float
    algo: int | None
    algos: np.ndarray | None
    lengths: np.ndarray
    messages: np.ndarray
    offsets: np.ndarray


def serving_requests(n_requests: int, rate_per_s: float, seed: int = 5, max_count: int = 10_000,
                     median: float = 256.0, sigma: float = 1.5, cap: int = 1 << 16,
                     mixed_fraction: float = 0.0) -> list[Request]:
    """Open-loop Poisson arrivals at rate_per_s.  Message count per request is log-uniform
    on [1, max_count]; algorithm uniform over the three; lengths log-normal (median 256 B,
    sigma 1.5, cap 64 KiB).  A fraction mixed_fraction of requests mixes algorithms per
    message."""
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    t = np.cumsum(gaps)
    out = []
    for r in range(n_requests):
        cnt = int(np.clip(np.floor(np.exp(rng.uniform(0.0, np.log(max_count + 1)))), 1, max_count))
        lens = lognormal_lengths(rng, cnt, median, sigma, cap)
        algo = int(rng.integers(0, 3))
        algos = None
        if mixed_fraction > 0 and rng.uniform() < mixed_fraction:
            algos = rng.integers(0, 3, size=cnt, dtype=np.uint8)
            algo = None
        offs = packed(lens)
        msgs = host_random_bytes(int(lens.sum()), seed * 1_000_003 + r)
        out.append(Request(float(t[r]), algo, algos, lens, msgs, offs))
    return out
