"""Pins for the CPU oracle: checks against facts fixed outside the oracle itself.

* the standards' own worked examples (tests/golden/standard_vectors.tsv);
* an independent implementation (OpenSSL via hashlib) over every message length
  0..300 -- every residue mod 64 across five block counts -- and long messages;
* closed forms of the MD5 sine table (RFC 1321 Sec. 3.4) in 50-digit arithmetic and of
  the SHA-1 constants (integer square roots);
* the padding rule (RFC 1321 Sec. 3.1-3.2, FIPS 180-4 Sec. 5.1.1, GB/T 32905 Sec. 5.2)
  and the block count nb(L) = floor((L + 8) / 64) + 1;
* chain invariants: hashing the padded message block by block equals one-shot hashing.
"""
import hashlib
from pathlib import Path

import mpmath
import numpy as np
import pytest

from paper_2407_09333_amd import workloads

GOLDEN = Path(__file__).resolve().parent / "golden" / "standard_vectors.tsv"
NAMES = ("md5", "sha1", "sm3")


def _vectors():
    rows = []
    for line in GOLDEN.read_text().splitlines():
        if not line or line.startswith("#"):
            continue
        algo, rep, text, digest, src = line.split("\t")
        rows.append((algo, int(rep), text, digest, src))
    return rows


@pytest.mark.parametrize("algo,rep,text,digest,src", _vectors())
def test_standard_worked_examples(oracle_lib, algo, rep, text, digest, src):
    msg = text.encode("ascii") * rep
    assert oracle_lib.hash_one(algo, msg).hex() == digest, src
    # the fixture itself agrees with an independent implementation
    assert hashlib.new(algo, msg).hexdigest() == digest, src


def test_standard_vectors_cover_each_algorithm():
    algos = {r[0] for r in _vectors()}
    assert algos == set(NAMES)


@pytest.mark.parametrize("algo", NAMES)
def test_every_length_0_to_300_matches_openssl(oracle_lib, algo):
    buf = workloads.host_random_bytes(300, seed=11).tobytes()
    for L in range(301):
        assert oracle_lib.hash_one(algo, buf[:L]) == hashlib.new(algo, buf[:L]).digest(), L


@pytest.mark.parametrize("algo", NAMES)
@pytest.mark.parametrize("L", [0, 1, 55, 56, 63, 64, 119, 120, 127, 128, 183, 184, 1023, 1024, 1025])
def test_padding_edge_lengths(oracle_lib, algo, L):
    msg = workloads.host_random_bytes(L, seed=1000 + L).tobytes()
    assert oracle_lib.hash_one(algo, msg) == hashlib.new(algo, msg).digest()


@pytest.mark.parametrize("algo", NAMES)
def test_long_messages_match_openssl(oracle_lib, algo):
    for L, seed in ((1 << 20, 21), ((1 << 20) + 3, 22), (1_000_003, 23)):
        msg = workloads.host_random_bytes(L, seed=seed).tobytes()
        assert oracle_lib.hash_one(algo, msg) == hashlib.new(algo, msg).digest(), L


@pytest.mark.parametrize("L,nb", [(0, 1), (55, 1), (56, 2), (63, 2), (64, 2), (119, 2), (120, 3),
                                  (1024, 17), (4096, 65), (1 << 20, 16385)])
def test_block_count_formula(oracle_lib, L, nb):
    # nb(L) = floor((L + 8) / 64) + 1 blocks; padded length = 64 * nb
    assert (L + 8) // 64 + 1 == nb
    assert oracle_lib.padded_length(L) == 64 * nb


@pytest.mark.parametrize("algo", NAMES)
@pytest.mark.parametrize("L", [0, 3, 55, 56, 64, 100, 1000])
def test_padding_layout(oracle_lib, algo, L):
    msg = workloads.host_random_bytes(L, seed=77).tobytes()
    p = oracle_lib.pad(algo, msg)
    assert len(p) % 64 == 0 and len(p) >= L + 9 and len(p) - (L + 9) < 64
    assert p[:L] == msg
    assert p[L] == 0x80
    assert set(p[L + 1:-8]) <= {0}
    order = "little" if algo == "md5" else "big"
    assert int.from_bytes(p[-8:], order) == 8 * L


def test_md5_sine_table_closed_form(oracle_lib):
    # RFC 1321 Sec. 3.4: T[i] = floor(4294967296 * |sin(i)|), evaluated in 50 digits
    mpmath.mp.dps = 50
    want = [int(mpmath.floor(4294967296 * abs(mpmath.sin(i)))) for i in range(1, 65)]
    assert oracle_lib.md5_T().tolist() == want
    # first and last entries as the RFC tabulates them
    assert oracle_lib.md5_T()[0] == 0xD76AA478 and oracle_lib.md5_T()[63] == 0xEB86D391


def test_sha1_constants_closed_form(oracle_lib):
    import math

    K = oracle_lib.sha1_K().tolist()
    for k, c in zip(K, (2, 3, 5, 10)):
        assert k == math.isqrt(c << 60)
        assert k * k <= c << 60 < (k + 1) * (k + 1)
    # FIPS 180-4 Sec. 4.2.1
    assert K == [0x5A827999, 0x6ED9EBA1, 0x8F1BBCDC, 0xCA62C1D6]


@pytest.mark.parametrize("algo", NAMES)
def test_block_chain_equals_one_shot(oracle_lib, algo):
    msg = workloads.host_random_bytes(300, seed=5).tobytes()
    p = oracle_lib.pad(algo, msg)
    s = oracle_lib.initial_state(algo)
    for i in range(0, len(p), 64):
        s = oracle_lib.compress(algo, s, p[i:i + 64])
    order = "<u4" if algo == "md5" else ">u4"
    assert s.astype(order).tobytes() == oracle_lib.hash_one(algo, msg)
    assert oracle_lib.hash_padded(algo, p) == oracle_lib.hash_one(algo, msg)


def test_initial_values(oracle_lib):
    # RFC 1321 Sec. 3.3; FIPS 180-4 Sec. 5.3.1; GB/T 32905-2016 Sec. 4.1
    assert oracle_lib.initial_state("md5").tolist() == [0x67452301, 0xEFCDAB89, 0x98BADCFE, 0x10325476]
    assert oracle_lib.initial_state("sha1").tolist()[4] == 0xC3D2E1F0
    assert oracle_lib.initial_state("sm3").tolist()[0] == 0x7380166F


def test_sm3_expansion_shape(oracle_lib):
    # W'_j = W_j xor W_{j+4} (GB/T 32905 Sec. 5.3.2), W_0..W_15 are the big-endian words
    block = workloads.host_random_bytes(64, seed=9).tobytes()
    W, Wp = oracle_lib.sm3_expand(block)
    assert W[:16].tolist() == list(np.frombuffer(block, ">u4"))
    assert np.array_equal(Wp, W[:64] ^ W[4:68])


def test_batch_driver_matches_single(oracle_lib):
    b = workloads.uniform_lengths_batch(2, 500, 300, seed=8)
    # overlapping, unaligned extra message
    offs = np.concatenate([b.offsets, np.array([3], np.uint64)])
    lens = np.concatenate([b.lengths, np.array([200], np.uint64)])
    for algo in NAMES:
        out1 = oracle_lib.hash_batch(algo, b.messages, offs, lens, threads=1)
        out4 = oracle_lib.hash_batch(algo, b.messages, offs, lens, threads=4)
        assert np.array_equal(out1, out4)
        for i in range(offs.size):
            m = b.messages[int(offs[i]):int(offs[i] + lens[i])].tobytes()
            assert out1[i].tobytes() == hashlib.new(algo, m).digest()


def test_mixed_batch_driver(oracle_lib):
    b = workloads.mixed_batch(200_000, seed=4, cap=1 << 14)
    out = oracle_lib.hash_batch(b.algos, b.messages, b.offsets, b.lengths)
    assert out.shape == (b.n, 32)
    for i in range(0, b.n, 7):
        a = NAMES[int(b.algos[i])]
        m = b.messages[int(b.offsets[i]):int(b.offsets[i] + b.lengths[i])].tobytes()
        d = hashlib.new(a, m).digest()
        assert out[i, :len(d)].tobytes() == d
        assert not out[i, len(d):].any()


def test_batch_rejects_bad_algo(oracle_lib):
    with pytest.raises(ValueError):
        oracle_lib.hash_batch(7, np.zeros(4, np.uint8), np.zeros(1, np.uint64), np.ones(1, np.uint64))
