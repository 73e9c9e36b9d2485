"""Thin ctypes binding of libhb (declared in include/hb.h).

Argument marshalling only: every hashing step runs in the HIP library.  Device buffers are
torch CUDA tensors (uint8 messages, int64 offsets/lengths holding byte counts < 2^63);
the stream is torch's current stream unless one is given.  If libhb.so is missing the
binding raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import re
from pathlib import Path

import numpy as np

from . import DIGEST_SIZE, MD5, SHA1, SM3

PKG = Path(__file__).resolve().parent
LIB_PATH = PKG / "libhb.so"
HEADER = PKG.parent / "include" / "hb.h"

HB_OK, HB_EINVAL, HB_ENOMEM, HB_EHIP, HB_EBUDGET, HB_EBUSY, HB_ECANCELED = 0, -1, -2, -3, -4, -5, -6
PLAN_GRAPH, PLAN_AUTOTUNE, PLAN_NO_SORT, PLAN_NO_LONG, PLAN_LONG_INLINE = 1, 2, 4, 8, 16
ALGO_IDS = {"md5": MD5, "sha1": SHA1, "sm3": SM3}

_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64
_i = ctypes.c_int


class HBError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libhb status {status}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load libhb.so (built by paper_2407_09333_amd.build); raise if it is absent."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise ImportError(f"{LIB_PATH} is missing: run paper_2407_09333_amd.build.build() first")
        L = ctypes.CDLL(str(LIB_PATH))
        L.hb_digest_size.argtypes = [_i]
        L.hb_digest_size.restype = ctypes.c_size_t
        L.hb_last_error.restype = ctypes.c_char_p
        L.hb_device_info.argtypes = [ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i),
                                     ctypes.c_char_p, ctypes.c_size_t]
        if hasattr(L, "hb_probe_valu"):
            L.hb_probe_valu.argtypes = [_i, _i, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.hash_batch.argtypes = [_i, _vp, _vp, _vp, _u64, _vp, _vp]
        L.hash_batch_strided.argtypes = [_i, _vp, _vp, _vp, _u64, _vp, _u64, _vp]
        L.hash_batch_fixed.argtypes = [_i, _vp, _u64, _u64, _vp, _vp]
        L.hash_batch_mixed.argtypes = [_vp, _vp, _vp, _vp, _u64, _vp, _vp]
        L.hash_digits9.argtypes = [_i, _u64, _u64, _vp, _vp]
        L.hash_init_batch.argtypes = [_i, _vp, _u64, _vp]
        L.hash_update_batch.argtypes = [_i, _vp, _vp, _vp, _vp, _u64, _vp]
        L.hash_final_batch.argtypes = [_i, _vp, _vp, _vp, _vp, _u64, _vp, _vp]
        if hasattr(L, "hb_plan_create"):
            L.hb_plan_create.argtypes = [ctypes.POINTER(_vp), _u64, _i]
            L.hb_plan_run.argtypes = [_vp, _vp, _i, _vp, _vp, _vp, _u64, _vp, _vp]
            L.hb_plan_config.argtypes = [_vp, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i)]
            L.hb_plan_set_config.argtypes = [_vp, _i, _i, _i]
            L.hb_plan_kernel_ms.argtypes = [_vp]
            L.hb_plan_kernel_ms.restype = ctypes.c_double
            L.hb_plan_destroy.argtypes = [_vp]
            L.hb_plan_destroy.restype = None
        if hasattr(L, "hash_batch_bucketed_noalloc"):
            L.hash_batch_bucketed_noalloc.argtypes = [_vp, _i, _vp, _vp, _vp, _u64, _vp, _vp]
        if hasattr(L, "hash_batch_host"):
            L.hash_batch_host.argtypes = [_vp, _i, _vp, _vp, _vp, _u64, _vp, _u64]
        if hasattr(L, "hash_batch_host_split"):
            L.hash_batch_host_split.argtypes = [_vp, _i, _vp, _vp, _vp, _u64, _vp, _u64, ctypes.c_double, _i]
            L.hb_cpu_hash_batch.argtypes = [_vp, _i, _vp, _vp, _vp, _u64, _vp, _i]
        if hasattr(L, "hb_server_create"):
            L.hb_server_create.argtypes = [ctypes.POINTER(_vp), _i, _u64, _i]
            L.hb_server_submit.argtypes = [_vp, _i, _vp, _vp, _vp, _vp, _u64, _vp,
                                           ctypes.POINTER(_u64)]
            L.hb_server_poll.argtypes = [_vp, _u64, ctypes.POINTER(_i), ctypes.POINTER(_i)]
            L.hb_server_wait.argtypes = [_vp, _u64, ctypes.c_int64, ctypes.POINTER(_i)]
            L.hb_server_cancel.argtypes = [_vp, _u64]
            L.hb_server_release.argtypes = [_vp, _u64]
            L.hb_server_times.argtypes = [_vp, _u64] + [ctypes.POINTER(ctypes.c_double)] * 4
            L.hb_server_trace.argtypes = [_vp, _u64, ctypes.POINTER(ctypes.c_double), _i]
            L.hb_server_stats.argtypes = [_vp] + [ctypes.POINTER(_u64)] * 4
            L.hb_server_now.argtypes = [_vp]
            L.hb_server_now.restype = ctypes.c_double
            L.hb_server_destroy.argtypes = [_vp]
            L.hb_server_destroy.restype = None
        _lib = L
    return _lib


def declared_symbols() -> list[str]:
    """Function names declared in include/hb.h."""
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hb_\w+|hash_batch\w*)\s*\(", text)))


def last_error() -> str:
    return lib().hb_last_error().decode()


def check(status: int) -> int:
    if status != HB_OK:
        raise HBError(status, last_error())
    return status


def algo_id(a) -> int:
    return ALGO_IDS[a] if isinstance(a, str) else int(a)


def digest_size(algo) -> int:
    return int(lib().hb_digest_size(algo_id(algo)))


def device_info() -> dict:
    cu, ws, clk = _i(), _i(), _i()
    name = ctypes.create_string_buffer(64)
    check(lib().hb_device_info(ctypes.byref(cu), ctypes.byref(ws), ctypes.byref(clk), name, 64))
    return {"cu_count": cu.value, "wave_size": ws.value, "clock_khz": clk.value,
            "arch": name.value.decode()}


# hb_probe_valu kinds, in the order of include/hb.h
PROBE_KINDS = ["add3", "alignbit", "bitop3", "add", "xor", "xad", "perm", "mix_bitop3_alignbit_1_1",
               "mix_bitop3_alignbit_2_1", "md5", "sha1", "sm3"]


def probe_valu(kind: str, waves_per_simd: int = 4) -> tuple[float, float]:
    """SIMD cycles per wave instruction (per wave and block for the compression kinds) and
    the engine clock in GHz, from hb_probe_valu."""
    c, g = ctypes.c_double(), ctypes.c_double()
    check(lib().hb_probe_valu(PROBE_KINDS.index(kind), waves_per_simd, ctypes.byref(c), ctypes.byref(g)))
    return c.value, g.value


# ---------------------------------------------------------------------------------------
# torch marshalling helpers
# ---------------------------------------------------------------------------------------

def _torch():
    import torch

    return torch


def _stream_ptr(stream) -> int | None:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _dev_u8(x):
    torch = _torch()
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.uint8).reshape(-1))
    if not x.is_cuda:
        x = x.cuda()
    assert x.dtype == torch.uint8 and x.is_contiguous()
    return x


def _dev_i64(x):
    torch = _torch()
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x).astype(np.int64, copy=False).reshape(-1))
    if not x.is_cuda:
        x = x.cuda()
    assert x.dtype == torch.int64 and x.is_contiguous()
    return x


def _ptr(t) -> int | None:
    return t.data_ptr() if t is not None else None


def hash_batch(algo, messages, offsets, lengths, out=None, stride: int | None = None, stream=None):
    """Plain batch hashing; returns an (n, stride) uint8 CUDA tensor of digests."""
    torch = _torch()
    a = algo_id(algo)
    msgs, offs, lens = _dev_u8(messages), _dev_i64(offsets), _dev_i64(lengths)
    n = offs.numel()
    ds = DIGEST_SIZE.get(a, 32)
    stride = stride or ds
    if out is None:
        out = torch.empty((n, stride), dtype=torch.uint8, device=msgs.device)
    check(lib().hash_batch_strided(a, _ptr(msgs), _ptr(offs), _ptr(lens), n, _ptr(out), stride,
                                   _stream_ptr(stream)))
    return out


def hash_batch_fixed(algo, messages, n: int, msg_len: int, out=None, stream=None):
    """n contiguous messages of msg_len bytes; returns (n, digest) uint8 CUDA tensor."""
    torch = _torch()
    a = algo_id(algo)
    msgs = _dev_u8(messages)
    assert msgs.numel() >= n * msg_len
    if out is None:
        out = torch.empty((n, DIGEST_SIZE.get(a, 32)), dtype=torch.uint8, device=msgs.device)
    check(lib().hash_batch_fixed(a, _ptr(msgs), n, msg_len, _ptr(out), _stream_ptr(stream)))
    return out


def hash_batch_mixed(algos, messages, offsets, lengths, out=None, stream=None):
    """Per-message algorithm ids, plain form (one launch per algorithm); (n, 32) digests."""
    torch = _torch()
    al, msgs, offs, lens = _dev_u8(algos), _dev_u8(messages), _dev_i64(offsets), _dev_i64(lengths)
    n = offs.numel()
    if out is None:
        out = torch.empty((n, 32), dtype=torch.uint8, device=msgs.device)
    check(lib().hash_batch_mixed(_ptr(al), _ptr(msgs), _ptr(offs), _ptr(lens), n, _ptr(out),
                                 _stream_ptr(stream)))
    return out


def hash_digits9(algo, start: int, n: int, out=None, stream=None):
    """Digests of the 9-digit decimal strings of start .. start + n - 1 (generated on the
    device); returns an (n, digest) uint8 CUDA tensor."""
    torch = _torch()
    a = algo_id(algo)
    if out is None:
        out = torch.empty((n, DIGEST_SIZE.get(a, 32)), dtype=torch.uint8, device="cuda")
    check(lib().hash_digits9(a, start, n, _ptr(out), _stream_ptr(stream)))
    return out


STATE_BYTES = 48  # sizeof(hb_state): 8 chaining words, u64 byte count, u64 flags


def hash_init(algo, n: int, stream=None):
    """n chaining states (an (n, 6) int64 CUDA tensor, 48 bytes each) at the initial value."""
    torch = _torch()
    st = torch.empty((n, STATE_BYTES // 8), dtype=torch.int64, device="cuda")
    check(lib().hash_init_batch(algo_id(algo), _ptr(st), n, _stream_ptr(stream)))
    return st


def hash_update(algo, states, messages, offsets, lengths, stream=None):
    """Absorb whole-block pieces into the states (in place)."""
    msgs, offs, lens = _dev_u8(messages), _dev_i64(offsets), _dev_i64(lengths)
    check(lib().hash_update_batch(algo_id(algo), _ptr(states), _ptr(msgs), _ptr(offs), _ptr(lens),
                                  offs.numel(), _stream_ptr(stream)))
    return states


def hash_final(algo, states, messages, offsets, lengths, out=None, stream=None):
    """Absorb the last pieces and the padding; returns (n, digest) digests."""
    torch = _torch()
    a = algo_id(algo)
    msgs, offs, lens = _dev_u8(messages), _dev_i64(offsets), _dev_i64(lengths)
    n = offs.numel()
    if out is None:
        out = torch.empty((n, DIGEST_SIZE.get(a, 32)), dtype=torch.uint8, device="cuda")
    check(lib().hash_final_batch(a, _ptr(states), _ptr(msgs), _ptr(offs), _ptr(lens), n, _ptr(out),
                                 _stream_ptr(stream)))
    return out


class Plan:
    """Batched form: bucketed, longest-first persistent launch captured in a hipGraph."""

    def __init__(self, max_n: int, flags: int = PLAN_GRAPH):
        self._h = _vp()
        check(lib().hb_plan_create(ctypes.byref(self._h), max_n, flags))
        self.max_n = max_n

    def run(self, messages, offsets, lengths, algo=None, algos=None, out=None, stream=None):
        torch = _torch()
        msgs, offs, lens = _dev_u8(messages), _dev_i64(offsets), _dev_i64(lengths)
        n = offs.numel()
        al = _dev_u8(algos) if algos is not None else None
        a = algo_id(algo) if algo is not None else 0
        stride = 32 if al is not None else DIGEST_SIZE.get(a, 32)
        if out is None:
            out = torch.empty((n, stride), dtype=torch.uint8, device=msgs.device)
        check(lib().hb_plan_run(self._h, _ptr(al), a, _ptr(msgs), _ptr(offs), _ptr(lens), n,
                                _ptr(out), _stream_ptr(stream)))
        return out

    def config(self) -> dict:
        w, m, v = _i(), _i(), _i()
        check(lib().hb_plan_config(self._h, ctypes.byref(w), ctypes.byref(m), ctypes.byref(v)))
        return {"waves_per_cu": w.value, "msgs_per_lane": m.value, "variant": v.value}

    def set_config(self, waves_per_cu: int = 0, msgs_per_lane: int = 0, variant: int = 0):
        check(lib().hb_plan_set_config(self._h, waves_per_cu, msgs_per_lane, variant))

    def kernel_ms(self) -> float:
        return float(lib().hb_plan_kernel_ms(self._h))

    def close(self):
        if self._h:
            lib().hb_plan_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


NOALLOC_MAX_N = 1 << 20  # the static workspace's message limit (include/hb.h)


def hash_batch_bucketed_noalloc(messages, offsets, lengths, algo=None, algos=None, out=None, stream=None):
    """Batched form without a plan or any allocation in the library
    (hash_batch_bucketed_noalloc); digests as Plan.run."""
    torch = _torch()
    msgs, offs, lens = _dev_u8(messages), _dev_i64(offsets), _dev_i64(lengths)
    n = offs.numel()
    al = _dev_u8(algos) if algos is not None else None
    a = algo_id(algo) if algo is not None else 0
    stride = 32 if al is not None else DIGEST_SIZE.get(a, 32)
    if out is None:
        out = torch.empty((n, stride), dtype=torch.uint8, device=msgs.device)
    check(lib().hash_batch_bucketed_noalloc(_ptr(al), a, _ptr(msgs), _ptr(offs), _ptr(lens), n, _ptr(out),
                                            _stream_ptr(stream)))
    return out


def hash_batch_host(messages: np.ndarray, offsets: np.ndarray, lengths: np.ndarray, algo=None,
                    algos: np.ndarray | None = None, chunk_bytes: int = 64 << 20) -> np.ndarray:
    """Host-resident inputs: chunked H2D copies overlapped with hashing (zero-copy for small
    batches); numpy digests."""
    msgs, offs, lens, al, a, out = _host_args(messages, offsets, lengths, algo, algos)
    check(lib().hash_batch_host(al.ctypes.data if al is not None else None, a,
                                msgs.ctypes.data if msgs.size else None, offs.ctypes.data,
                                lens.ctypes.data, offs.size, out.ctypes.data, chunk_bytes))
    return out[: offs.size]


def _host_args(messages, offsets, lengths, algo, algos):
    msgs = np.ascontiguousarray(messages, dtype=np.uint8).reshape(-1)
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    lens = np.ascontiguousarray(lengths, dtype=np.uint64)
    al = np.ascontiguousarray(algos, dtype=np.uint8) if algos is not None else None
    a = algo_id(algo) if algo is not None else 0
    stride = 32 if al is not None else DIGEST_SIZE.get(a, 32)
    out = np.zeros((max(offs.size, 1), stride), np.uint8)
    return msgs, offs, lens, al, a, out


def hash_batch_host_split(messages: np.ndarray, offsets: np.ndarray, lengths: np.ndarray, algo=None,
                          algos: np.ndarray | None = None, cpu_fraction: float = 0.0, cpu_threads: int = 0,
                          chunk_bytes: int = 64 << 20) -> np.ndarray:
    """CPU + GPU split of a host-resident batch (hash_batch_host_split); numpy digests."""
    msgs, offs, lens, al, a, out = _host_args(messages, offsets, lengths, algo, algos)
    check(lib().hash_batch_host_split(al.ctypes.data if al is not None else None, a,
                                      msgs.ctypes.data if msgs.size else None, offs.ctypes.data,
                                      lens.ctypes.data, offs.size, out.ctypes.data, chunk_bytes,
                                      float(cpu_fraction), int(cpu_threads)))
    return out[: offs.size]


def cpu_hash_batch(messages: np.ndarray, offsets: np.ndarray, lengths: np.ndarray, algo=None,
                   algos: np.ndarray | None = None, threads: int = 0) -> np.ndarray:
    """The host-core share's hashing on its own (hb_cpu_hash_batch); numpy digests."""
    msgs, offs, lens, al, a, out = _host_args(messages, offsets, lengths, algo, algos)
    check(lib().hb_cpu_hash_batch(al.ctypes.data if al is not None else None, a,
                                  msgs.ctypes.data if msgs.size else None, offs.ctypes.data,
                                  lens.ctypes.data, offs.size, out.ctypes.data, int(threads)))
    return out[: offs.size]


class Server:
    """Continuous-batching serving loop (hb_server_*).  Requests are host numpy buffers,
    kept alive here until they complete."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 256, device: int = 0):
        self._h = _vp()
        check(lib().hb_server_create(ctypes.byref(self._h), device, hbm_budget_bytes, max_slots))
        self._live = {}
        self._trace_raw = None

    def submit(self, messages: np.ndarray, offsets: np.ndarray, lengths: np.ndarray, algo=None,
               algos: np.ndarray | None = None) -> int:
        msgs = np.ascontiguousarray(messages, dtype=np.uint8).reshape(-1)
        offs = np.ascontiguousarray(offsets, dtype=np.uint64)
        lens = np.ascontiguousarray(lengths, dtype=np.uint64)
        al = np.ascontiguousarray(algos, dtype=np.uint8) if algos is not None else None
        a = -1 if al is not None else algo_id(algo)
        stride = 32 if al is not None else DIGEST_SIZE.get(a, 32)
        out = np.zeros((max(offs.size, 1), stride), np.uint8)
        t = _u64()
        check(lib().hb_server_submit(self._h, a, al.ctypes.data if al is not None else None,
                                     msgs.ctypes.data if msgs.size else None, offs.ctypes.data,
                                     lens.ctypes.data, offs.size, out.ctypes.data, ctypes.byref(t)))
        self._live[t.value] = (msgs, offs, lens, al, out)
        return t.value

    def poll(self, ticket: int):
        d, st = _i(), _i()
        check(lib().hb_server_poll(self._h, ticket, ctypes.byref(d), ctypes.byref(st)))
        return bool(d.value), st.value

    def wait(self, ticket: int, timeout_ms: int = -1) -> np.ndarray:
        """Digests of a finished request; raises HBError with the request's status if it
        failed or was cancelled (HB_EBUSY on timeout)."""
        st = _i()
        check(lib().hb_server_wait(self._h, ticket, timeout_ms, ctypes.byref(st)))
        msgs, offs, lens, al, out = self._live.pop(ticket)
        check(st.value)
        return out[: offs.size]

    def cancel(self, ticket: int) -> bool:
        """Cancel a request not yet admitted (True); False once it has been admitted."""
        rc = lib().hb_server_cancel(self._h, ticket)
        if rc == HB_EBUSY:
            return False
        check(rc)
        return True

    def release(self, ticket: int):
        """Drop a finished request's record (its status, times and trace)."""
        check(lib().hb_server_release(self._h, ticket))
        self._live.pop(ticket, None)

    def times(self, ticket: int) -> dict:
        v = [ctypes.c_double() for _ in range(4)]
        check(lib().hb_server_times(self._h, ticket, *[ctypes.byref(x) for x in v]))
        return dict(zip(("submit", "admit", "h2d_done", "done"), (x.value for x in v)))

    TRACE_NAMES = ("submit", "admit", "stage_begin", "stage_end", "h2d_done", "launch", "exec_begin",
                   "exec_end", "done")

    def trace(self, ticket: int) -> dict:
        """Per-request timestamps (hb_server_trace), keyed by TRACE_NAMES."""
        v = (ctypes.c_double * len(self.TRACE_NAMES))()
        check(lib().hb_server_trace(self._h, ticket, v, len(self.TRACE_NAMES)))
        return dict(zip(self.TRACE_NAMES, list(v)))

    def collect(self, ticket: int, trace_out: np.ndarray) -> None:
        """Wait for a request, write its trace (TRACE_NAMES order) into trace_out (a C-contiguous
        float64 array of len(TRACE_NAMES)) and release it, with no digest copy or dict built:
        the low-overhead path for a client that consumes results as they finish.  Raises
        HBError with the request's status if it failed (after releasing it)."""
        assert trace_out.dtype == np.float64 and trace_out.size >= len(self.TRACE_NAMES) and trace_out.flags.c_contiguous
        if self._trace_raw is None:
            self._trace_raw = lib()["hb_server_trace"]  # a second prototype taking a plain address
            self._trace_raw.argtypes = [_vp, _u64, _vp, _i]
        st = _i()
        check(lib().hb_server_wait(self._h, ticket, -1, ctypes.byref(st)))
        self._live.pop(ticket, None)
        rc = self._trace_raw(self._h, ticket, trace_out.ctypes.data, len(self.TRACE_NAMES))
        check(lib().hb_server_release(self._h, ticket))
        check(rc)
        check(st.value)

    def stats(self) -> dict:
        v = [_u64() for _ in range(4)]
        check(lib().hb_server_stats(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("completed", "steps", "stalls", "peak_bytes"), (x.value for x in v)))

    def now(self) -> float:
        return float(lib().hb_server_now(self._h))

    def close(self):
        if self._h:
            lib().hb_server_destroy(self._h)
            self._h = _vp()
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
