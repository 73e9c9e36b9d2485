/*
 * hash_oracle.c -- plain, slow, obviously-correct CPU reference for MD5, SHA-1 and SM3.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this
 * file: only the test suite, the smoke check and the benchmark's CPU-baseline leg do.
 * It shares no code, header, table or generator with the HIP implementation.
 *
 * The paper (batch hashing of many independent messages, Sec. IV-B "parallel scenario"
 * crypto ops and Sec. V-A.2 data preparation) names the three algorithms but does not
 * define them, so every function below follows the defining standard:
 *   MD5   -- RFC 1321 Sec. 3.1-3.5
 *   SHA-1 -- FIPS 180-4 Sec. 4.1.1, 4.2.1, 5.1.1, 5.2.1, 5.3.1, 6.1.2
 *   SM3   -- GB/T 32905-2016 Sec. 4.1-4.4, 5.2, 5.3.2, 5.3.3, 5.4
 *
 * Method: the whole padded message is materialised in host memory (Sec. 3.1-3.2 /
 * 5.1.1 / 5.2), split into 64-byte blocks, each block decoded into 16 words, and the
 * compression function applied block by block in the standard's order and notation.
 * No blocking, fusion or reordering beyond the standards' own definitions.
 *
 * Pins (see tests/test_oracle_*.py): the standards' worked examples, an independent
 * library (OpenSSL through Python's hashlib) over every length 0..300 and long
 * messages, closed forms of the MD5 sine table and the SHA-1 square-root constants,
 * and split invariants of the block chain.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MD5 0
#define ORACLE_SHA1 1
#define ORACLE_SM3 2

/* --------------------------------------------------------------------------------- */
/* Common helpers                                                                     */
/* --------------------------------------------------------------------------------- */

/* Circular left shift of a 32-bit word by s positions, 0 <= s < 32.  Written so that
 * s == 0 never evaluates x >> 32 (undefined in C); SM3 reaches s == 0 at j == 32. */
static uint32_t rotl32(uint32_t x, unsigned s)
{
    s &= 31u;
    if (s == 0) return x;
    return (x << s) | (x >> (32u - s));
}

static uint32_t load_le32(const uint8_t *p)
{
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

static uint32_t load_be32(const uint8_t *p)
{
    return ((uint32_t)p[0] << 24) | ((uint32_t)p[1] << 16) | ((uint32_t)p[2] << 8) | (uint32_t)p[3];
}

static void store_le32(uint8_t *p, uint32_t v)
{
    p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); p[2] = (uint8_t)(v >> 16); p[3] = (uint8_t)(v >> 24);
}

static void store_be32(uint8_t *p, uint32_t v)
{
    p[0] = (uint8_t)(v >> 24); p[1] = (uint8_t)(v >> 16); p[2] = (uint8_t)(v >> 8); p[3] = (uint8_t)v;
}

int oracle_digest_size(int algo)
{
    switch (algo) {
    case ORACLE_MD5: return 16;
    case ORACLE_SHA1: return 20;
    case ORACLE_SM3: return 32;
    default: return 0;
    }
}

/* Padded length in bytes: the message, one 0x80 byte, k zero bytes and an 8-byte length
 * field, rounded to the next multiple of 64 (RFC 1321 Sec. 3.1-3.2, FIPS 180-4 Sec. 5.1.1,
 * GB/T 32905-2016 Sec. 5.2).  The smallest total >= len + 9 that is a multiple of 64. */
uint64_t oracle_padded_length(uint64_t len)
{
    uint64_t need = len + 9u;
    return (need + 63u) / 64u * 64u;
}

/* Write the padded message into out[0 .. oracle_padded_length(len)).
 * Step 1: copy the message.  Step 2: append the single '1' bit, as byte 0x80 (messages
 * here are whole bytes).  Step 3: append zero bytes up to 56 mod 64.  Step 4: append the
 * bit length as a 64-bit integer -- low-order byte first for MD5 (RFC 1321 Sec. 3.2),
 * high-order byte first for SHA-1 (FIPS 180-4 Sec. 5.1.1) and SM3 (GB/T 32905 Sec. 5.2). */
int oracle_pad(int algo, const uint8_t *msg, uint64_t len, uint8_t *out)
{
    uint64_t total = oracle_padded_length(len);
    uint64_t bits = len * 8u;
    if (oracle_digest_size(algo) == 0) return -1;
    if (len) memcpy(out, msg, (size_t)len);
    out[len] = 0x80;
    memset(out + len + 1, 0, (size_t)(total - 8 - len - 1));
    for (int i = 0; i < 8; i++) {
        uint8_t b = (uint8_t)(bits >> (8 * i));
        if (algo == ORACLE_MD5)
            out[total - 8 + i] = b;          /* little-endian */
        else
            out[total - 1 - i] = b;          /* big-endian */
    }
    return 0;
}

/* --------------------------------------------------------------------------------- */
/* MD5 (RFC 1321)                                                                     */
/* --------------------------------------------------------------------------------- */

/* Sec. 3.4: T[i] is the integer part of 4294967296 * abs(sin(i)), i in radians, i=1..64.
 * Computed here from that definition rather than typed in. */
static uint32_t md5_T[65];
static int md5_T_ready = 0;

static void md5_make_table(void)
{
    if (md5_T_ready) return;
    for (int i = 1; i <= 64; i++)
        md5_T[i] = (uint32_t)floor(4294967296.0 * fabs(sin((double)i)));
    md5_T_ready = 1;
}

void oracle_md5_T(uint32_t out[64])
{
    md5_make_table();
    for (int i = 0; i < 64; i++) out[i] = md5_T[i + 1];
}

/* Sec. 3.4 auxiliary functions. */
static uint32_t md5_F(uint32_t x, uint32_t y, uint32_t z) { return (x & y) | (~x & z); }
static uint32_t md5_G(uint32_t x, uint32_t y, uint32_t z) { return (x & z) | (y & ~z); }
static uint32_t md5_H(uint32_t x, uint32_t y, uint32_t z) { return x ^ y ^ z; }
static uint32_t md5_I(uint32_t x, uint32_t y, uint32_t z) { return y ^ (x | ~z); }

/* Sec. 3.4: one 16-word block X[0..15].  Each of the 64 operations has the form
 *   a = b + ((a + Fn(b,c,d) + X[k] + T[i]) <<< s)
 * where the round r = 0..3 fixes Fn (F, G, H, I), the shifts and the word order;
 * after each operation the roles of (a,b,c,d) rotate right by one, as in the standard's
 * listing [ABCD] [DABC] [CDAB] [BCDA].  Word order per round for operation j = 0..15:
 *   round 1: j;  round 2: (1 + 5j) mod 16;  round 3: (5 + 3j) mod 16;  round 4: 7j mod 16. */
void oracle_md5_compress(uint32_t state[4], const uint8_t block[64])
{
    static const unsigned shifts[4][4] = {
        {7, 12, 17, 22}, {5, 9, 14, 20}, {4, 11, 16, 23}, {6, 10, 15, 21}};
    uint32_t X[16];
    md5_make_table();
    for (int j = 0; j < 16; j++) X[j] = load_le32(block + 4 * j);   /* Sec. 3.4: LE words */

    uint32_t v[4] = {state[0], state[1], state[2], state[3]};       /* AA=A, BB=B, ... */
    for (int i = 0; i < 64; i++) {
        int r = i / 16, j = i % 16, k;
        uint32_t f;
        /* positions of a, b, c, d in v[] for operation i: a slot moves back by one each op */
        int ia = (4 - (i % 4)) % 4, ib = (ia + 1) % 4, ic = (ia + 2) % 4, id = (ia + 3) % 4;
        uint32_t b = v[ib], c = v[ic], d = v[id];
        switch (r) {
        case 0: f = md5_F(b, c, d); k = j; break;
        case 1: f = md5_G(b, c, d); k = (1 + 5 * j) % 16; break;
        case 2: f = md5_H(b, c, d); k = (5 + 3 * j) % 16; break;
        default: f = md5_I(b, c, d); k = (7 * j) % 16; break;
        }
        v[ia] = b + rotl32(v[ia] + f + X[k] + md5_T[i + 1], shifts[r][i % 4]);
    }
    for (int q = 0; q < 4; q++) state[q] += v[q];                    /* A = A + AA, ... */
}

/* Sec. 3.3: the registers as the standard writes them, low-order bytes first:
 * A = 01 23 45 67, B = 89 ab cd ef, C = fe dc ba 98, D = 76 54 32 10. */
static void md5_init(uint32_t s[4])
{
    static const uint8_t iv_bytes[16] = {0x01, 0x23, 0x45, 0x67, 0x89, 0xab, 0xcd, 0xef,
                                         0xfe, 0xdc, 0xba, 0x98, 0x76, 0x54, 0x32, 0x10};
    for (int i = 0; i < 4; i++) s[i] = load_le32(iv_bytes + 4 * i);
}

/* --------------------------------------------------------------------------------- */
/* SHA-1 (FIPS 180-4)                                                                 */
/* --------------------------------------------------------------------------------- */

/* Integer square root: the largest r with r*r <= v (bit-by-bit method). */
static uint64_t isqrt_u64(uint64_t v)
{
    uint64_t r = 0, bit = (uint64_t)1 << 62;
    while (bit > v) bit >>= 2;
    while (bit) {
        if (v >= r + bit) { v -= r + bit; r = (r >> 1) + bit; }
        else r >>= 1;
        bit >>= 2;
    }
    return r;
}

/* Sec. 4.2.1 lists K_t as four hex constants; they are the integer parts of
 * 2^30 * sqrt(2), sqrt(3), sqrt(5), sqrt(10), i.e. isqrt(c * 2^60), computed exactly. */
void oracle_sha1_K(uint32_t out[4])
{
    static const uint64_t c[4] = {2, 3, 5, 10};
    for (int i = 0; i < 4; i++) out[i] = (uint32_t)isqrt_u64(c[i] << 60);
}

/* Sec. 4.1.1: Ch, Parity, Maj. */
static uint32_t sha1_f(int t, uint32_t x, uint32_t y, uint32_t z)
{
    if (t < 20) return (x & y) ^ (~x & z);            /* Ch */
    if (t < 40) return x ^ y ^ z;                      /* Parity */
    if (t < 60) return (x & y) ^ (x & z) ^ (y & z);    /* Maj */
    return x ^ y ^ z;                                  /* Parity */
}

/* Sec. 6.1.2 steps 1-4 for one block M^(i). */
void oracle_sha1_compress(uint32_t H[5], const uint8_t block[64])
{
    uint32_t W[80], K[4];
    oracle_sha1_K(K);
    /* 1. message schedule */
    for (int t = 0; t < 16; t++) W[t] = load_be32(block + 4 * t);
    for (int t = 16; t < 80; t++) W[t] = rotl32(W[t - 3] ^ W[t - 8] ^ W[t - 14] ^ W[t - 16], 1);
    /* 2. working variables */
    uint32_t a = H[0], b = H[1], c = H[2], d = H[3], e = H[4];
    /* 3. eighty rounds */
    for (int t = 0; t < 80; t++) {
        uint32_t T = rotl32(a, 5) + sha1_f(t, b, c, d) + e + K[t / 20] + W[t];
        e = d;
        d = c;
        c = rotl32(b, 30);
        b = a;
        a = T;
    }
    /* 4. intermediate hash value */
    H[0] += a; H[1] += b; H[2] += c; H[3] += d; H[4] += e;
}

/* Sec. 5.3.1: initial hash value. */
static void sha1_init(uint32_t H[5])
{
    H[0] = 0x67452301u; H[1] = 0xefcdab89u; H[2] = 0x98badcfeu; H[3] = 0x10325476u; H[4] = 0xc3d2e1f0u;
}

/* --------------------------------------------------------------------------------- */
/* SM3 (GB/T 32905-2016)                                                              */
/* --------------------------------------------------------------------------------- */

/* Sec. 4.2 constants T_j. */
static uint32_t sm3_T(int j) { return j <= 15 ? 0x79cc4519u : 0x7a879d8au; }

/* Sec. 4.3 Boolean functions. */
static uint32_t sm3_FF(int j, uint32_t X, uint32_t Y, uint32_t Z)
{
    return j <= 15 ? (X ^ Y ^ Z) : ((X & Y) | (X & Z) | (Y & Z));
}
static uint32_t sm3_GG(int j, uint32_t X, uint32_t Y, uint32_t Z)
{
    return j <= 15 ? (X ^ Y ^ Z) : ((X & Y) | (~X & Z));
}

/* Sec. 4.4 permutations. */
static uint32_t sm3_P0(uint32_t X) { return X ^ rotl32(X, 9) ^ rotl32(X, 17); }
static uint32_t sm3_P1(uint32_t X) { return X ^ rotl32(X, 15) ^ rotl32(X, 23); }

/* Sec. 5.3.2 message expansion: W_0..W_67 and W'_0..W'_63. */
void oracle_sm3_expand(const uint8_t block[64], uint32_t W[68], uint32_t Wp[64])
{
    for (int j = 0; j < 16; j++) W[j] = load_be32(block + 4 * j);
    for (int j = 16; j < 68; j++)
        W[j] = sm3_P1(W[j - 16] ^ W[j - 9] ^ rotl32(W[j - 3], 15)) ^ rotl32(W[j - 13], 7) ^ W[j - 6];
    for (int j = 0; j < 64; j++) Wp[j] = W[j] ^ W[j + 4];
}

/* Sec. 5.3.3 compression function CF(V_i, B_i); V_{i+1} = CF(V_i, B_i) (Sec. 5.3.1). */
void oracle_sm3_compress(uint32_t V[8], const uint8_t block[64])
{
    uint32_t W[68], Wp[64];
    oracle_sm3_expand(block, W, Wp);
    uint32_t A = V[0], B = V[1], C = V[2], D = V[3], E = V[4], F = V[5], G = V[6], H = V[7];
    for (int j = 0; j < 64; j++) {
        uint32_t SS1 = rotl32(rotl32(A, 12) + E + rotl32(sm3_T(j), (unsigned)(j % 32)), 7);
        uint32_t SS2 = SS1 ^ rotl32(A, 12);
        uint32_t TT1 = sm3_FF(j, A, B, C) + D + SS2 + Wp[j];
        uint32_t TT2 = sm3_GG(j, E, F, G) + H + SS1 + W[j];
        D = C;
        C = rotl32(B, 9);
        B = A;
        A = TT1;
        H = G;
        G = rotl32(F, 19);
        F = E;
        E = sm3_P0(TT2);
    }
    /* V_{i+1} = ABCDEFGH xor V_i */
    V[0] ^= A; V[1] ^= B; V[2] ^= C; V[3] ^= D; V[4] ^= E; V[5] ^= F; V[6] ^= G; V[7] ^= H;
}

/* Sec. 4.1 initial value IV. */
static void sm3_init(uint32_t V[8])
{
    V[0] = 0x7380166fu; V[1] = 0x4914b2b9u; V[2] = 0x172442d7u; V[3] = 0xda8a0600u;
    V[4] = 0xa96f30bcu; V[5] = 0x163138aau; V[6] = 0xe38dee4du; V[7] = 0xb0fb0e4eu;
}

/* --------------------------------------------------------------------------------- */
/* One message                                                                        */
/* --------------------------------------------------------------------------------- */

/* Chain the compression function over the blocks of an already padded message and
 * write the digest: MD5 registers low-order byte first (RFC 1321 Sec. 3.5), SHA-1 and
 * SM3 words high-order byte first (FIPS 180-4 Sec. 6.1.2; GB/T 32905 Sec. 5.4). */
int oracle_hash_padded(int algo, const uint8_t *padded, uint64_t nblocks, uint8_t *out)
{
    uint32_t s[8];
    switch (algo) {
    case ORACLE_MD5:
        md5_init(s);
        for (uint64_t i = 0; i < nblocks; i++) oracle_md5_compress(s, padded + 64 * i);
        for (int q = 0; q < 4; q++) store_le32(out + 4 * q, s[q]);
        return 0;
    case ORACLE_SHA1:
        sha1_init(s);
        for (uint64_t i = 0; i < nblocks; i++) oracle_sha1_compress(s, padded + 64 * i);
        for (int q = 0; q < 5; q++) store_be32(out + 4 * q, s[q]);
        return 0;
    case ORACLE_SM3:
        sm3_init(s);
        for (uint64_t i = 0; i < nblocks; i++) oracle_sm3_compress(s, padded + 64 * i);
        for (int q = 0; q < 8; q++) store_be32(out + 4 * q, s[q]);
        return 0;
    default:
        return -1;
    }
}

/* Initial chaining value of each algorithm as words (for split-chain tests). */
int oracle_initial_state(int algo, uint32_t *s)
{
    switch (algo) {
    case ORACLE_MD5: md5_init(s); return 4;
    case ORACLE_SHA1: sha1_init(s); return 5;
    case ORACLE_SM3: sm3_init(s); return 8;
    default: return -1;
    }
}

int oracle_compress(int algo, uint32_t *s, const uint8_t block[64])
{
    switch (algo) {
    case ORACLE_MD5: oracle_md5_compress(s, block); return 0;
    case ORACLE_SHA1: oracle_sha1_compress(s, block); return 0;
    case ORACLE_SM3: oracle_sm3_compress(s, block); return 0;
    default: return -1;
    }
}

/* Digest of one message of len bytes: pad, then chain over the blocks. */
int oracle_hash(int algo, const uint8_t *msg, uint64_t len, uint8_t *out)
{
    if (oracle_digest_size(algo) == 0) return -1;
    uint64_t total = oracle_padded_length(len);
    uint8_t stackbuf[1024];
    uint8_t *buf = total <= sizeof stackbuf ? stackbuf : (uint8_t *)malloc((size_t)total);
    if (!buf) return -2;
    oracle_pad(algo, msg, len, buf);
    int rc = oracle_hash_padded(algo, buf, total / 64, out);
    if (buf != stackbuf) free(buf);
    return rc;
}

/* --------------------------------------------------------------------------------- */
/* Many messages (the paper's multi-message "parallel scenario", Sec. IV-B)            */
/* --------------------------------------------------------------------------------- */

/* Message i is base[offsets[i] .. offsets[i] + lengths[i]); its digest goes to
 * out + i * out_stride (bytes past the digest size are left untouched).  algos == NULL
 * hashes every message with `algo`; otherwise message i uses algos[i].  The messages are
 * independent (separate input and output slots, Sec. V-D), so they are spread over
 * nthreads host threads (0 = the OpenMP default) with a dynamic schedule.
 * Returns 0, -1 for an invalid algorithm id, -2 on allocation failure. */
static int batch_impl(const uint8_t *algos, int algo, const uint8_t *base, const uint64_t *offsets,
                      const uint64_t *lengths, uint64_t n, uint8_t *out, uint64_t out_stride,
                      int nthreads)
{
    int rc = 0;
    md5_make_table(); /* build the shared table before the threads start */
    for (uint64_t i = 0; algos && i < n; i++)
        if (oracle_digest_size(algos[i]) == 0) return -1;
    if (!algos && oracle_digest_size(algo) == 0) return -1;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads) reduction(min : rc)
#endif
    for (int64_t i = 0; i < (int64_t)n; i++) {
        int a = algos ? algos[i] : algo;
        int r = oracle_hash(a, base + offsets[i], lengths[i], out + (uint64_t)i * out_stride);
        if (r < rc) rc = r;
    }
    (void)nthreads;
    return rc;
}

int oracle_hash_batch(int algo, const uint8_t *base, const uint64_t *offsets, const uint64_t *lengths,
                      uint64_t n, uint8_t *out, uint64_t out_stride, int nthreads)
{
    return batch_impl(NULL, algo, base, offsets, lengths, n, out, out_stride, nthreads);
}

int oracle_hash_batch_mixed(const uint8_t *algos, const uint8_t *base, const uint64_t *offsets,
                            const uint64_t *lengths, uint64_t n, uint8_t *out, uint64_t out_stride,
                            int nthreads)
{
    return batch_impl(algos, 0, base, offsets, lengths, n, out, out_stride, nthreads);
}

/* Number of threads the batch driver uses for nthreads <= 0. */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
