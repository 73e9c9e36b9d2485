"""The integer-VALU issue-rate probe (hb_probe_valu) behind the roofline's peak: it runs on
every kind, its figures are consistent with the op-mix model the bench prices the kernels
with, and it rejects bad arguments."""
import math

import pytest

pytestmark = pytest.mark.gpu

# (full-rate, half-rate) ops per block, as the roofline counts them
OPS_BY_RATE = {"md5": (196, 128), "sha1": (213, 400), "sm3": (484, 864)}


@pytest.fixture(scope="module")
def hb():
    import torch

    assert torch.cuda.is_available()
    from paper_2407_09333_amd import hb as _hb

    return _hb


def test_probe_every_kind(hb):
    for k in hb.PROBE_KINDS:
        print(f"case probe kind={k}", flush=True)
        c, g = hb.probe_valu(k, 4)
        assert math.isfinite(c) and c > 0, k
        assert 0.5 < g < 4.0, (k, g)  # the engine clock in GHz


def test_probe_rates_match_the_op_mix_model(hb):
    """v_bitop3_b32 issues at about twice v_add3_u32's rate with several waves per SIMD;
    no compression issues faster than the op-mix model allows (2 cycles per full-rate op,
    4 per half-rate op, per wave and block)."""
    print("case probe rates", flush=True)
    add3 = hb.probe_valu("add3", 8)[0]
    bitop3 = hb.probe_valu("bitop3", 8)[0]
    assert 3.5 < add3 < 5.0
    assert bitop3 < 0.75 * add3
    for a, (full, half) in OPS_BY_RATE.items():
        c = hb.probe_valu(a, 4)[0]
        assert c > 0.95 * (2 * full + 4 * half), (a, c)


def test_probe_rejects_bad_arguments(hb):
    from paper_2407_09333_amd.hb import HB_EINVAL, HBError, lib
    import ctypes

    c = ctypes.c_double()
    assert lib().hb_probe_valu(len(hb.PROBE_KINDS), 4, ctypes.byref(c), None) == HB_EINVAL
    assert lib().hb_probe_valu(0, 0, ctypes.byref(c), None) == HB_EINVAL
    assert lib().hb_probe_valu(0, 9, ctypes.byref(c), None) == HB_EINVAL
    assert lib().hb_probe_valu(0, 4, None, None) == HB_EINVAL
    with pytest.raises(HBError):
        hb.probe_valu("add3", 0)
