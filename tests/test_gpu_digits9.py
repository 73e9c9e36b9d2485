"""The paper's own workload (Sec. V-A.2): digests of the 9-character decimal strings,
generated on the device.  The oracle hashes the same strings built on the host by the
input generator."""
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


@pytest.mark.parametrize("algo", [0, 1, 2])
@pytest.mark.parametrize("start,n", [(0, 1000), (999_999_000, 1000), (123_456_789, 70_001)])
def test_digits9_matches_oracle(hb, algo, start, n):
    print(f"case digits9 algo={algo} start={start} n={n}", flush=True)
    b = workloads.digits9_batch(n, start=start)
    got = hb.hash_digits9(algo, start, n).cpu().numpy()
    assert_same(got, oracle.hash_batch(algo, b.messages, b.offsets, b.lengths), "digits9")


def test_digits9_first_and_last_strings(hb):
    import hashlib

    for algo, name in ((0, "md5"), (1, "sha1"), (2, "sm3")):
        first = hb.hash_digits9(algo, 0, 1).cpu().numpy()[0].tobytes()
        last = hb.hash_digits9(algo, 999_999_999, 1).cpu().numpy()[0].tobytes()
        assert first == oracle.hash_one(algo, b"000000000")
        assert last == oracle.hash_one(algo, b"999999999")
        assert first == hashlib.new(name, b"000000000").digest()
