"""C-ABI contract checks that need no GPU: the library loads, exports every symbol that
include/hb.h declares, and rejects malformed arguments before touching a device."""
import ctypes

import pytest

from paper_2407_09333_amd import hb


@pytest.fixture(scope="module")
def L():
    return hb.lib()


def test_every_declared_symbol_is_exported(L):
    names = hb.declared_symbols()
    assert "hash_batch" in names and "hb_plan_run" in names and "hb_server_submit" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_digest_sizes(L):
    assert [hb.digest_size(a) for a in (0, 1, 2)] == [16, 20, 32]
    assert hb.digest_size(3) == 0 and hb.digest_size(-1) == 0


def test_bad_algo_rejected_before_launch(L):
    rc = L.hash_batch(7, None, None, None, 10, None, None)
    assert rc == hb.HB_EINVAL
    assert "algorithm" in hb.last_error()


def test_n_zero_is_noop(L):
    assert L.hash_batch(0, None, None, None, 0, None, None) == hb.HB_OK
    assert L.hash_batch_fixed(2, None, 0, 64, None, None) == hb.HB_OK
    assert L.hash_batch_mixed(None, None, None, None, 0, None, None) == hb.HB_OK


def test_null_pointers_rejected(L):
    assert L.hash_batch(1, None, None, None, 5, None, None) == hb.HB_EINVAL
    assert L.hash_batch(1, 16, None, None, 5, 64, None) == hb.HB_EINVAL  # null offsets
    assert L.hash_batch_mixed(None, 16, 16, 16, 5, 64, None) == hb.HB_EINVAL


def test_misaligned_output_and_bad_stride_rejected(L):
    assert L.hash_batch_strided(0, 16, 16, 16, 5, 66, 16, None) == hb.HB_EINVAL
    assert L.hash_batch_strided(2, 16, 16, 16, 5, 64, 20, None) == hb.HB_EINVAL  # < 32
    assert L.hash_batch_strided(1, 16, 16, 16, 5, 64, 22, None) == hb.HB_EINVAL  # not /4


def test_fixed_length_limit(L):
    assert L.hash_batch_fixed(0, 16, 4, 1 << 61, 64, None) == hb.HB_EINVAL


def test_last_error_is_thread_local(L):
    import threading

    L.hash_batch(9, None, None, None, 1, None, None)
    seen = {}

    def other():
        seen["msg"] = hb.last_error()

    t = threading.Thread(target=other)
    t.start()
    t.join()
    assert seen["msg"] == ""
    assert "algorithm" in hb.last_error()


def test_digits9_range_checked_before_launch(L):
    assert L.hash_digits9(0, 999_999_999, 2, 64, None) == hb.HB_EINVAL
    assert L.hash_digits9(0, 1_000_000_000, 1, 64, None) == hb.HB_EINVAL
    assert L.hash_digits9(5, 0, 10, 64, None) == hb.HB_EINVAL
    assert L.hash_digits9(1, 0, 0, None, None) == hb.HB_OK


def test_state_layout_and_stream_argument_checks(L):
    import ctypes

    assert hb.STATE_BYTES == 48
    assert L.hash_init_batch(9, 64, 1, None) == hb.HB_EINVAL
    assert L.hash_init_batch(0, None, 3, None) == hb.HB_EINVAL
    assert L.hash_init_batch(0, 68, 3, None) == hb.HB_EINVAL  # not 8-byte aligned
    assert L.hash_update_batch(1, 64, None, None, None, 2, None) == hb.HB_EINVAL
    assert L.hash_final_batch(2, 64, 64, 64, 64, 2, 66, None) == hb.HB_EINVAL  # misaligned out
    assert L.hash_final_batch(2, None, None, None, None, 0, None, None) == hb.HB_OK
