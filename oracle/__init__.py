"""CPU oracle for batch hashing (MD5, SHA-1, SM3) -- test infrastructure only.

The shared library ``liboracle.so`` is built from ``hash_oracle.c`` (plain C written
from RFC 1321, FIPS 180-4 and GB/T 32905-2016).  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path never does, and
the two implementations share no code.

Every function takes and returns plain numpy arrays / bytes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

MD5, SHA1, SM3 = 0, 1, 2
ALGOS = {"md5": MD5, "sha1": SHA1, "sm3": SM3}
DIGEST_SIZE = {MD5: 16, SHA1: 20, SM3: 32}

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "hash_oracle.c"
_LIB = _HERE / "liboracle.so"

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = True) -> Path:
    """Compile hash_oracle.c with gcc (-O2, OpenMP) into liboracle.so."""
    if force or not _LIB.exists():
        tmp = _LIB.with_suffix(".so.tmp")
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-fopenmp",
               str(_SRC), "-o", str(tmp), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not _LIB.exists():
            build()
        L = ctypes.CDLL(str(_LIB))
        L.oracle_digest_size.argtypes = [ctypes.c_int]
        L.oracle_padded_length.argtypes = [ctypes.c_uint64]
        L.oracle_padded_length.restype = ctypes.c_uint64
        L.oracle_pad.argtypes = [ctypes.c_int, _u8p, ctypes.c_uint64, _u8p]
        L.oracle_hash.argtypes = [ctypes.c_int, _u8p, ctypes.c_uint64, _u8p]
        L.oracle_hash_padded.argtypes = [ctypes.c_int, _u8p, ctypes.c_uint64, _u8p]
        L.oracle_initial_state.argtypes = [ctypes.c_int, _u32p]
        L.oracle_compress.argtypes = [ctypes.c_int, _u32p, _u8p]
        L.oracle_md5_T.argtypes = [_u32p]
        L.oracle_sha1_K.argtypes = [_u32p]
        L.oracle_sm3_expand.argtypes = [_u8p, _u32p, _u32p]
        L.oracle_hash_batch.argtypes = [ctypes.c_int, _u8p, _u64p, _u64p, ctypes.c_uint64, _u8p,
                                        ctypes.c_uint64, ctypes.c_int]
        L.oracle_hash_batch_mixed.argtypes = [_u8p, _u8p, _u64p, _u64p, ctypes.c_uint64, _u8p,
                                              ctypes.c_uint64, ctypes.c_int]
        L.oracle_max_threads.argtypes = []
        _lib = L
    return _lib


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def _u8(data) -> np.ndarray:
    if isinstance(data, np.ndarray):
        return np.ascontiguousarray(data, dtype=np.uint8).reshape(-1)
    return np.frombuffer(bytes(data), dtype=np.uint8)


def _algo(a) -> int:
    return ALGOS[a] if isinstance(a, str) else int(a)


def digest_size(algo) -> int:
    return lib().oracle_digest_size(_algo(algo))


def hash_one(algo, msg) -> bytes:
    """Digest of one message (RFC 1321 / FIPS 180-4 / GB/T 32905)."""
    a = _algo(algo)
    m = _u8(msg)
    buf = m if m.size else np.zeros(1, np.uint8)
    out = np.zeros(32, np.uint8)
    rc = lib().oracle_hash(a, _ptr(buf, _u8p), m.size, _ptr(out, _u8p))
    if rc != 0:
        raise ValueError(f"oracle_hash failed ({rc}) for algo {algo!r}")
    return out[: DIGEST_SIZE[a]].tobytes()


def pad(algo, msg) -> bytes:
    """The padded message (message, 0x80, zeros, 64-bit bit length)."""
    a = _algo(algo)
    m = _u8(msg)
    buf = m if m.size else np.zeros(1, np.uint8)
    out = np.zeros(int(lib().oracle_padded_length(m.size)), np.uint8)
    if lib().oracle_pad(a, _ptr(buf, _u8p), m.size, _ptr(out, _u8p)) != 0:
        raise ValueError("bad algo")
    return out.tobytes()


def padded_length(n: int) -> int:
    return int(lib().oracle_padded_length(n))


def initial_state(algo) -> np.ndarray:
    s = np.zeros(8, np.uint32)
    k = lib().oracle_initial_state(_algo(algo), _ptr(s, _u32p))
    if k < 0:
        raise ValueError("bad algo")
    return s[:k].copy()


def compress(algo, state: np.ndarray, block) -> np.ndarray:
    """One application of the compression function; returns the new chaining value."""
    s = np.zeros(8, np.uint32)
    s[: state.size] = state
    b = _u8(block)
    assert b.size == 64
    lib().oracle_compress(_algo(algo), _ptr(s, _u32p), _ptr(b, _u8p))
    return s[: state.size].copy()


def hash_padded(algo, padded) -> bytes:
    a = _algo(algo)
    p = _u8(padded)
    assert p.size % 64 == 0 and p.size > 0
    out = np.zeros(32, np.uint8)
    lib().oracle_hash_padded(a, _ptr(p, _u8p), p.size // 64, _ptr(out, _u8p))
    return out[: DIGEST_SIZE[a]].tobytes()


def md5_T() -> np.ndarray:
    t = np.zeros(64, np.uint32)
    lib().oracle_md5_T(_ptr(t, _u32p))
    return t


def sha1_K() -> np.ndarray:
    k = np.zeros(4, np.uint32)
    lib().oracle_sha1_K(_ptr(k, _u32p))
    return k


def sm3_expand(block):
    b = _u8(block)
    W = np.zeros(68, np.uint32)
    Wp = np.zeros(64, np.uint32)
    lib().oracle_sm3_expand(_ptr(b, _u8p), _ptr(W, _u32p), _ptr(Wp, _u32p))
    return W, Wp


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def hash_batch(algo, messages: np.ndarray, offsets: np.ndarray, lengths: np.ndarray,
               out_stride: int | None = None, threads: int = 0) -> np.ndarray:
    """Digests of many messages; returns an (n, out_stride) uint8 array (zero-filled
    beyond each digest).  algo may be an int/str, or a uint8 array of per-message ids."""
    msgs = _u8(messages)
    if msgs.size == 0:
        msgs = np.zeros(1, np.uint8)
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    lens = np.ascontiguousarray(lengths, dtype=np.uint64)
    n = offs.size
    assert lens.size == n
    mixed = isinstance(algo, np.ndarray)
    if out_stride is None:
        out_stride = 32 if mixed else DIGEST_SIZE.get(_algo(algo), 32)
    out = np.zeros((max(n, 1), out_stride), np.uint8)
    if n:
        assert int((offs + lens).max()) <= msgs.size or int(lens.max()) == 0
    if mixed:
        al = np.ascontiguousarray(algo, dtype=np.uint8)
        assert al.size == n
        rc = lib().oracle_hash_batch_mixed(_ptr(al, _u8p), _ptr(msgs, _u8p), _ptr(offs, _u64p),
                                           _ptr(lens, _u64p), n, _ptr(out, _u8p), out_stride,
                                           threads)
    else:
        rc = lib().oracle_hash_batch(_algo(algo), _ptr(msgs, _u8p), _ptr(offs, _u64p),
                                     _ptr(lens, _u64p), n, _ptr(out, _u8p), out_stride, threads)
    if rc != 0:
        raise ValueError(f"oracle batch failed ({rc})")
    return out[:n]
