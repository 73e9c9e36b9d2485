"""MI355X-native batch hashing (MD5, SHA-1, SM3) over very many independent messages.

The compute path is the HIP library ``libhb.so`` (hand-written gfx950 kernels behind a
C ABI, declared in ``include/hb.h``); :mod:`paper_2407_09333_amd.hb` is its thin ctypes
binding.  PyTorch only provides device memory and streams.
"""
MD5, SHA1, SM3 = 0, 1, 2
ALGO_NAMES = {MD5: "md5", SHA1: "sha1", SM3: "sm3"}
DIGEST_SIZE = {MD5: 16, SHA1: 20, SM3: 32}
