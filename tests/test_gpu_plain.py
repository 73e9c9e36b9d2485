"""Parity of the plain HIP path (hash_batch / hash_batch_fixed / hash_batch_mixed) with
the CPU oracle: every digest bit-exact on the same seeded inputs."""
import numpy as np
import pytest

import oracle
from paper_2407_09333_amd import workloads
from tests.gpu_util import assert_same, check_guard, guarded_out, to_dev

pytestmark = pytest.mark.gpu

ALGOS = [0, 1, 2]


@pytest.fixture(scope="module")
def hb():
    import torch

    assert torch.cuda.is_available()
    from paper_2407_09333_amd import hb as _hb

    return _hb


def test_md5_4096_by_55(hb):
    b = workloads.cfg_md5_4096x55()
    print("case md5 4096x55", flush=True)
    got = hb.hash_batch_fixed(0, b.messages, b.n, 55).cpu().numpy()
    want = oracle.hash_batch(0, b.messages, b.offsets, b.lengths)
    assert_same(got, want, "md5 4096x55")


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("L", [0, 1, 3, 4, 9, 55, 56, 63, 64, 65, 119, 120, 127, 128, 200, 1023, 1024, 1029])
def test_fixed_lengths(hb, algo, L):
    n = 300  # ragged: not a multiple of the 256-lane workgroup
    b = workloads.fixed_batch(algo, n, L, seed=100 + L)
    print(f"case fixed algo={algo} L={L}", flush=True)
    msgs = b.messages if b.messages.size else np.zeros(1, np.uint8)
    got = hb.hash_batch_fixed(algo, msgs, n, L).cpu().numpy()
    assert_same(got, oracle.hash_batch(algo, b.messages, b.offsets, b.lengths), f"fixed L={L}")


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("n,L", [(300, 1024), (640, 128), (1000, 4), (515, 132), (4096, 2048), (128, 1028),
                                 (257, 256), (64, 60), (320, 384), (200, 640), (256, 512), (96, 768),
                                 (192, 896), (130, 1152)])
def test_fixed_lds_staged(hb, monkeypatch, algo, n, L):
    """The LDS-staged fixed-length kernel (the default; set explicitly): whole waves stage
    two blocks per burst through LDS, partial waves and the last blocks go per lane; burst
    counts 0 to 9 and 16, lengths with and without a padding-only last block; digests
    bit-exact against the oracle, and no write outside the digest buffer."""
    monkeypatch.setenv("HB_PLAIN_LDS", "1")
    b = workloads.fixed_batch(algo, n, L, seed=500 + L)
    print(f"case fixed lds algo={algo} n={n} L={L}", flush=True)
    ds = oracle.DIGEST_SIZE[algo]
    buf, out = guarded_out(n, ds)
    hb.hash_batch_fixed(algo, b.messages, n, L, out=out)
    check_guard(buf, n, ds)
    assert_same(out.cpu().numpy(), oracle.hash_batch(algo, b.messages, b.offsets, b.lengths), "fixed lds")


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("shift", [4, 8, 12])
@pytest.mark.parametrize("L", [1024, 1028])
def test_fixed_lds_staged_base_off_16_bytes(hb, algo, shift, L):
    """A fixed-length batch whose buffer starts 4, 8 or 12 bytes past a 16-byte boundary (a
    view into a larger device buffer): the LDS-staged kernel's 16-byte buffer loads fall on
    dword-aligned addresses only; digests bit-exact against the oracle."""
    import torch

    n = 200
    b = workloads.fixed_batch(algo, n, L, seed=900 + shift + L)
    big = torch.zeros(n * L + 64, dtype=torch.uint8, device="cuda")
    big[shift:shift + n * L] = torch.from_numpy(b.messages).cuda()
    view = big[shift:shift + n * L]
    assert view.data_ptr() % 16 == shift
    print(f"case fixed lds shifted base algo={algo} shift={shift} L={L}", flush=True)
    ds = oracle.DIGEST_SIZE[algo]
    buf, out = guarded_out(n, ds)
    hb.hash_batch_fixed(algo, view, n, L, out=out)
    check_guard(buf, n, ds)
    assert_same(out.cpu().numpy(), oracle.hash_batch(algo, b.messages, b.offsets, b.lengths), "fixed lds shifted")


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("n,L", [(300, 1024), (515, 132), (320, 384), (64, 60)])
def test_fixed_per_lane(hb, monkeypatch, algo, n, L):
    """Fixed-length batches with HB_PLAIN_LDS=0 take the per-lane kernel (the LDS-staged one
    is the default): the same digests, bit-exact against the oracle."""
    monkeypatch.setenv("HB_PLAIN_LDS", "0")
    b = workloads.fixed_batch(algo, n, L, seed=800 + L)
    print(f"case fixed per-lane algo={algo} n={n} L={L}", flush=True)
    ds = oracle.DIGEST_SIZE[algo]
    buf, out = guarded_out(n, ds)
    hb.hash_batch_fixed(algo, b.messages, n, L, out=out)
    check_guard(buf, n, ds)
    assert_same(out.cpu().numpy(), oracle.hash_batch(algo, b.messages, b.offsets, b.lengths), "fixed per-lane")


@pytest.mark.parametrize("algo", ALGOS)
def test_every_length_0_to_300_packed(hb, algo):
    lens = np.arange(301, dtype=np.uint64)
    offs = workloads.packed(lens)
    msgs = workloads.host_random_bytes(int(lens.sum()), seed=31)
    print(f"case packed 0..300 algo={algo}", flush=True)
    ds = oracle.DIGEST_SIZE[algo]
    buf, out = guarded_out(lens.size, ds)
    hb.hash_batch(algo, msgs, offs, lens, out=out)
    check_guard(buf, lens.size, ds)
    assert_same(out.cpu().numpy(), oracle.hash_batch(algo, msgs, offs, lens), "packed 0..300")


# Lengths at and around the multi-block burst boundaries (whole blocks are read four at a
# time for MD5 and two at a time for SHA-1 / SM3, then one at a time, then the padded tail).
BURST_EDGES = sorted({64 * k + d for k in range(1, 11) for d in (-9, -8, -1, 0, 1)} | {1023, 1024, 1025, 4095, 4096})


@pytest.mark.parametrize("algo", ALGOS)
def test_burst_boundaries_every_alignment(hb, algo):
    """Every length around the burst boundaries, at byte offsets 0..7 (the realigning path
    and the aligned one), packed into one batch, plus the same lengths hashed by the
    bucketed plan."""
    lens, offs, pos = [], [], 0
    for r in range(8):
        for L in BURST_EDGES:
            pos += (r - pos) % 8  # next offset congruent to r mod 8
            offs.append(pos)
            lens.append(L)
            pos += L
    lens = np.array(lens, np.uint64)
    offs = np.array(offs, np.uint64)
    msgs = workloads.host_random_bytes(pos + 8, seed=47)
    print(f"case burst boundaries algo={algo} n={lens.size}", flush=True)
    want = oracle.hash_batch(algo, msgs, offs, lens)
    assert_same(hb.hash_batch(algo, msgs, offs, lens).cpu().numpy(), want, "burst edges plain")
    plan = hb.Plan(lens.size)
    assert_same(plan.run(msgs, offs, lens, algo=algo).cpu().numpy(), want, "burst edges plan")
    plan.close()


@pytest.mark.parametrize("algo", ALGOS)
def test_uneven_uniform_0_4096(hb, algo):
    b = workloads.uniform_lengths_batch(algo, 5000, 4096, seed=3)
    print(f"case uneven algo={algo}", flush=True)
    got = hb.hash_batch(algo, b.messages, b.offsets, b.lengths).cpu().numpy()
    assert_same(got, oracle.hash_batch(algo, b.messages, b.offsets, b.lengths), "uneven")


@pytest.mark.parametrize("algo", ALGOS)
def test_alignment_sweep_same_digest(hb, algo):
    base = workloads.host_random_bytes(1200, seed=44)
    msgs = np.concatenate([np.zeros(16, np.uint8), base, np.zeros(16, np.uint8)])
    # the same 1000-byte message placed at offsets 0..15 of a larger buffer
    buf = np.zeros(16 * 1100, np.uint8)
    offs = np.zeros(16, np.uint64)
    for r in range(16):
        o = r * 1100 + r
        buf[o:o + 1000] = base[:1000]
        offs[r] = o
    lens = np.full(16, 1000, np.uint64)
    print(f"case alignment algo={algo}", flush=True)
    got = hb.hash_batch(algo, buf, offs, lens).cpu().numpy()
    want = oracle.hash_one(algo, base[:1000])
    for r in range(16):
        assert got[r].tobytes() == want, r
    del msgs


@pytest.mark.parametrize("algo", ALGOS)
def test_overlapping_and_permuted_messages(hb, algo):
    data = workloads.host_random_bytes(5000, seed=45)
    rng = np.random.default_rng(7)
    offs = rng.integers(0, 2500, size=777).astype(np.uint64)
    lens = rng.integers(0, 2500, size=777).astype(np.uint64)
    print(f"case overlap algo={algo}", flush=True)
    got = hb.hash_batch(algo, data, offs, lens).cpu().numpy()
    assert_same(got, oracle.hash_batch(algo, data, offs, lens), "overlap")
    perm = rng.permutation(777)
    got2 = hb.hash_batch(algo, data, offs[perm], lens[perm]).cpu().numpy()
    assert_same(got2, got[perm], "permutation")


@pytest.mark.parametrize("algo", ALGOS)
def test_strided_output_zero_fills(hb, algo):
    b = workloads.uniform_lengths_batch(algo, 400, 300, seed=46)
    print(f"case strided algo={algo}", flush=True)
    buf, out = guarded_out(b.n, 36)
    hb.hash_batch(algo, b.messages, b.offsets, b.lengths, out=out, stride=36)
    check_guard(buf, b.n, 36)
    assert_same(out.cpu().numpy(), oracle.hash_batch(algo, b.messages, b.offsets, b.lengths, out_stride=36),
                "strided")


def test_mixed_plain(hb):
    b = workloads.mixed_batch(400_000, seed=4, cap=1 << 15)
    al = b.algos.copy()
    al[::97] = 9  # unknown ids leave an all-zero slot
    print(f"case mixed plain n={b.n}", flush=True)
    got = hb.hash_batch_mixed(al, b.messages, b.offsets, b.lengths).cpu().numpy()
    want = oracle.hash_batch(b.algos, b.messages, b.offsets, b.lengths)
    want[::97] = 0
    assert_same(got, want, "mixed plain")


def test_n_zero_and_one(hb):
    import torch

    out = torch.full((1, 32), 7, dtype=torch.uint8, device="cuda")
    msgs = workloads.host_random_bytes(100, seed=1)
    hb.hash_batch(2, msgs, np.zeros(0, np.uint64), np.zeros(0, np.uint64), out=out[:0])
    assert (out.cpu().numpy() == 7).all()
    got = hb.hash_batch(2, msgs, np.array([5], np.uint64), np.array([90], np.uint64)).cpu().numpy()
    assert got[0].tobytes() == oracle.hash_one(2, msgs[5:95])


@pytest.mark.parametrize("algo", ALGOS)
def test_full_size_fixed_1m_x_1024_all(hb, algo):
    """2^20 messages of 1,024 bytes in the bench's launch configuration; every one of the
    2^20 digests checked against the oracle (the whole 1 GiB buffer copied back and hashed
    on all host cores)."""
    import torch

    b = workloads.cfg_fixed_1m_x_1024(algo, device="cuda")
    print(f"case full fixed algo={algo}", flush=True)
    got = hb.hash_batch_fixed(algo, b.messages, b.n, 1024)
    torch.cuda.synchronize()
    host = b.messages.cpu().numpy()
    want = oracle.hash_batch(algo, host, b.offsets, b.lengths)
    assert_same(got.cpu().numpy(), want, "full fixed, every digest")


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("L,n", [((1 << 25) - 4, 65), (1 << 25, 64)])
def test_fixed_longest_messages_lds_limit(hb, algo, L, n):
    """Fixed-length messages at the LDS-staged kernel's length limit: 2^25 - 4 bytes is the
    longest it takes (the wave's 64 messages span 2^31 - 256 bytes, its buffer range; its
    32-bit load offsets reach 1.9 GB), with a partial second wave; 2^25 bytes goes to the
    per-lane kernel.  Every digest bit-exact against the oracle."""
    import torch

    msgs = workloads.host_random_bytes(n * L, seed=1300 + algo + (L & 7))
    offs = np.arange(n, dtype=np.uint64) * np.uint64(L)
    lens = np.full(n, L, np.uint64)
    print(f"case fixed longest algo={algo} L={L} n={n}", flush=True)
    dev = torch.from_numpy(msgs).cuda()
    ds = oracle.DIGEST_SIZE[algo]
    buf, out = guarded_out(n, ds)
    hb.hash_batch_fixed(algo, dev, n, L, out=out)
    check_guard(buf, n, ds)
    del dev
    assert_same(out.cpu().numpy(), oracle.hash_batch(algo, msgs, offs, lens), "fixed longest")
