"""Planted mistakes in a copy of the oracle must be caught by its pins.

Each case edits one plausible slip into a temporary copy of oracle/hash_oracle.c (a
dropped term, a wrong index, rotation or endianness, add instead of xor), compiles it on
the CPU and runs the same checks the pin tests use: the standards' worked examples and
OpenSSL over lengths 0..130.  The mutant must fail at least one of them.
"""
import ctypes
import hashlib
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
SRC = ROOT / "oracle" / "hash_oracle.c"
GOLDEN = Path(__file__).resolve().parent / "golden" / "standard_vectors.tsv"

MUTATIONS = {
    "md5_drop_T": ("+ md5_T[i + 1], shifts", ", shifts"),
    "md5_G_wrong": ("(x & z) | (y & ~z)", "(x & z) | (y & z)"),
    "md5_round2_index": ("(1 + 5 * j) % 16", "(1 + 3 * j) % 16"),
    "md5_shift_table": ("{5, 9, 14, 20}", "{5, 9, 14, 21}"),
    "md5_length_big_endian": ("if (algo == ORACLE_MD5)\n", "if (0)\n"),
    "sha1_rotl30": ("rotl32(b, 30)", "rotl32(b, 31)"),
    "sha1_schedule_term": ("^ W[t - 14] ", ""),
    "sha1_maj_as_ch": ("(x & y) ^ (x & z) ^ (y & z)", "(x & y) ^ (~x & z)"),
    "sha1_round_boundary": ("if (t < 40) return x ^ y ^ z;", "if (t < 41) return x ^ y ^ z;"),
    "sm3_chain_add": ("V[0] ^= A;", "V[0] += A;"),
    "sm3_wprime_index": ("W[j] ^ W[j + 4]", "W[j] ^ W[j + 3]"),
    "sm3_T_unrotated": ("rotl32(sm3_T(j), (unsigned)(j % 32))", "sm3_T(j)"),
    "sm3_P0_rotation": ("X ^ rotl32(X, 9) ^ rotl32(X, 17)", "X ^ rotl32(X, 9) ^ rotl32(X, 18)"),
    "sm3_GG_boundary": ("return j <= 15 ? (X ^ Y ^ Z) : ((X & Y) | (~X & Z));",
                        "return j <= 16 ? (X ^ Y ^ Z) : ((X & Y) | (~X & Z));"),
    "sm3_TT2_uses_Wprime": ("+ H + SS1 + W[j];", "+ H + SS1 + Wp[j];"),
    "pad_marker_byte": ("out[len] = 0x80;", "out[len] = 0x01;"),
    "pad_extra_block": ("(need + 63u) / 64u * 64u", "(need + 64u) / 64u * 64u"),
    "digest_endianness": ("for (int q = 0; q < 5; q++) store_be32", "for (int q = 0; q < 5; q++) store_le32"),
}


def _load(path):
    L = ctypes.CDLL(str(path))
    L.oracle_hash.argtypes = [ctypes.c_int, ctypes.c_char_p, ctypes.c_uint64, ctypes.c_char_p]
    return L


def _pins_pass(L) -> bool:
    ids = {"md5": 0, "sha1": 1, "sm3": 2}
    out = ctypes.create_string_buffer(32)
    for line in GOLDEN.read_text().splitlines():
        if not line or line.startswith("#"):
            continue
        algo, rep, text, digest, _ = line.split("\t")
        msg = text.encode() * int(rep)
        L.oracle_hash(ids[algo], msg, len(msg), out)
        if out.raw[: len(digest) // 2].hex() != digest:
            return False
    buf = bytes(range(131)) * 2
    for algo, a in ids.items():
        for n in range(131):
            m = buf[n:2 * n]
            L.oracle_hash(a, m, len(m), out)
            d = hashlib.new(algo, m).digest()
            if out.raw[: len(d)] != d:
                return False
    return True


@pytest.fixture(scope="module")
def workdir(tmp_path_factory):
    return tmp_path_factory.mktemp("oracle_mutants")


def _compile(src_text, d: Path, name: str) -> Path:
    c = d / f"{name}.c"
    so = d / f"{name}.so"
    c.write_text(src_text)
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-fopenmp", str(c), "-o", str(so), "-lm"],
                   check=True, capture_output=True)
    return so


def test_unmutated_copy_passes(workdir):
    assert _pins_pass(_load(_compile(SRC.read_text(), workdir, "orig")))


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(workdir, name):
    old, new = MUTATIONS[name]
    text = SRC.read_text()
    assert text.count(old) >= 1, f"mutation anchor not found: {old!r}"
    mutant = text.replace(old, new, 1)
    assert not _pins_pass(_load(_compile(mutant, workdir, name))), name
