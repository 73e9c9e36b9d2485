// hb_device.hpp -- per-lane MD5 / SHA-1 / SM3 cores for gfx950.
//
// One GPU lane owns one message.  Message words are read straight from HBM with
// dword-aligned global_load_dwordx4 and realigned (and, for the big-endian algorithms,
// byte-reversed) by one v_perm_b32 per word; the final one or two blocks -- tail bytes,
// the 0x80 marker, zeros and the 64-bit bit length (RFC 1321 Sec. 3.1-3.2, FIPS 180-4
// Sec. 5.1.1, GB/T 32905 Sec. 5.2) -- are assembled in registers, so no padded copy of
// the input ever exists.  The compression functions are fully unrolled with the state
// and message schedule in VGPRs, using v_alignbit_b32 rotates, v_bitop3_b32 for every
// three-input boolean function (including three-way xor) and v_add3_u32 / v_xad_u32 for
// the sums.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hb_md5_table.hpp"

namespace hb {

enum : int { MD5 = 0, SHA1 = 1, SM3 = 2 };

#define HB_GLOBAL __attribute__((address_space(1)))

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef u32x4 u32x4_a4 __attribute__((aligned(4)));  // 16-byte load needing only dword alignment

// ---------------------------------------------------------------------------------------
// Primitive operations
// ---------------------------------------------------------------------------------------

// Truth tables for v_bitop3_b32: bit k of the table is f(src0, src1, src2) where k =
// 4*src0 + 2*src1 + src2, i.e. f evaluated on the byte patterns 0xF0, 0xCC, 0xAA.
constexpr uint32_t tt_of(uint32_t v) { return v & 0xFFu; }
constexpr uint32_t TT_XOR3 = tt_of(0xF0u ^ 0xCCu ^ 0xAAu);                          // x^y^z
constexpr uint32_t TT_MAJ = tt_of((0xF0u & 0xCCu) | (0xF0u & 0xAAu) | (0xCCu & 0xAAu));
constexpr uint32_t TT_CH = tt_of((0xF0u & 0xCCu) | (~0xF0u & 0xAAu));                // (x&y)|(~x&z)
constexpr uint32_t TT_MD5_G = tt_of((0xF0u & 0xAAu) | (0xCCu & ~0xAAu));             // (x&z)|(y&~z)
constexpr uint32_t TT_MD5_I = tt_of(0xCCu ^ (0xF0u | ~0xAAu));                       // y^(x|~z)
static_assert(TT_XOR3 == 0x96 && TT_MAJ == 0xE8 && TT_CH == 0xCA, "bitop3 tables");

template <uint32_t TT>
__device__ __forceinline__ uint32_t bitop3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, TT);
}

// Left rotation by a compile-time amount 1..31: alignbit({x,x}, 32 - s).
template <uint32_t S>
__device__ __forceinline__ uint32_t rotl(uint32_t x)
{
    static_assert(S > 0 && S < 32, "rotation amount");
    return __builtin_amdgcn_alignbit(x, x, 32u - S);
}

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel)
{
    return __builtin_amdgcn_perm(hi, lo, sel);
}

__device__ __forceinline__ uint32_t bswap32(uint32_t x) { return perm(x, x, 0x00010203u); }

// v_perm selector extracting the 4 message bytes that start r bytes into {hi:lo}
// (hi = next dword).  Little-endian word for MD5, byte-reversed word for SHA-1 / SM3.
__device__ __forceinline__ uint32_t sel_le(uint32_t r) { return 0x03020100u + r * 0x01010101u; }
__device__ __forceinline__ uint32_t sel_be(uint32_t r) { return 0x00010203u + r * 0x01010101u; }

// ---------------------------------------------------------------------------------------
// Algorithm traits
// ---------------------------------------------------------------------------------------

template <int A> struct Traits;
template <> struct Traits<MD5> { static constexpr int kWords = 4, kDigest = 16; static constexpr bool kBE = false; };
template <> struct Traits<SHA1> { static constexpr int kWords = 5, kDigest = 20; static constexpr bool kBE = true; };
template <> struct Traits<SM3> { static constexpr int kWords = 8, kDigest = 32; static constexpr bool kBE = true; };

// ---------------------------------------------------------------------------------------
// MD5 (RFC 1321 Sec. 3.3-3.4)
// ---------------------------------------------------------------------------------------

__device__ __forceinline__ void md5_init(uint32_t s[8])
{
    s[0] = 0x67452301u; s[1] = 0xefcdab89u; s[2] = 0x98badcfeu; s[3] = 0x10325476u;
}

// One 64-step compression.  Step i: a = b + rotl(a + Fn(b,c,d) + X[k] + T_i, s), then
// (a,b,c,d) <- (d,a,b,c); Fn / k / s as in the RFC's four rounds.
__device__ __forceinline__ void md5_compress(uint32_t s[8], const uint32_t X[16])
{
    constexpr const uint32_t *T = kMd5T;
    uint32_t a = s[0], b = s[1], c = s[2], d = s[3];
#define HB_MD5_STEP(TTF, k, sh, i)                                           \
    {                                                                        \
        uint32_t t = a + bitop3<TTF>(b, c, d) + X[k] + T[i];                 \
        a = d; d = c; c = b;                                                 \
        b = b + rotl<sh>(t);                                                 \
    }
#pragma unroll
    for (int j = 0; j < 16; j += 4) {
        HB_MD5_STEP(TT_CH, j + 0, 7, j + 0)
        HB_MD5_STEP(TT_CH, j + 1, 12, j + 1)
        HB_MD5_STEP(TT_CH, j + 2, 17, j + 2)
        HB_MD5_STEP(TT_CH, j + 3, 22, j + 3)
    }
#pragma unroll
    for (int j = 0; j < 16; j += 4) {
        HB_MD5_STEP(TT_MD5_G, (1 + 5 * (j + 0)) & 15, 5, 16 + j + 0)
        HB_MD5_STEP(TT_MD5_G, (1 + 5 * (j + 1)) & 15, 9, 16 + j + 1)
        HB_MD5_STEP(TT_MD5_G, (1 + 5 * (j + 2)) & 15, 14, 16 + j + 2)
        HB_MD5_STEP(TT_MD5_G, (1 + 5 * (j + 3)) & 15, 20, 16 + j + 3)
    }
#pragma unroll
    for (int j = 0; j < 16; j += 4) {
        HB_MD5_STEP(TT_XOR3, (5 + 3 * (j + 0)) & 15, 4, 32 + j + 0)
        HB_MD5_STEP(TT_XOR3, (5 + 3 * (j + 1)) & 15, 11, 32 + j + 1)
        HB_MD5_STEP(TT_XOR3, (5 + 3 * (j + 2)) & 15, 16, 32 + j + 2)
        HB_MD5_STEP(TT_XOR3, (5 + 3 * (j + 3)) & 15, 23, 32 + j + 3)
    }
#pragma unroll
    for (int j = 0; j < 16; j += 4) {
        HB_MD5_STEP(TT_MD5_I, (7 * (j + 0)) & 15, 6, 48 + j + 0)
        HB_MD5_STEP(TT_MD5_I, (7 * (j + 1)) & 15, 10, 48 + j + 1)
        HB_MD5_STEP(TT_MD5_I, (7 * (j + 2)) & 15, 15, 48 + j + 2)
        HB_MD5_STEP(TT_MD5_I, (7 * (j + 3)) & 15, 21, 48 + j + 3)
    }
#undef HB_MD5_STEP
    s[0] += a; s[1] += b; s[2] += c; s[3] += d;
}

// ---------------------------------------------------------------------------------------
// SHA-1 (FIPS 180-4 Sec. 4.1.1, 4.2.1, 5.3.1, 6.1.2)
// ---------------------------------------------------------------------------------------

__device__ __forceinline__ void sha1_init(uint32_t s[8])
{
    s[0] = 0x67452301u; s[1] = 0xefcdab89u; s[2] = 0x98badcfeu; s[3] = 0x10325476u; s[4] = 0xc3d2e1f0u;
}

// 80 rounds over a 16-word rolling schedule W[t mod 16].
__device__ __forceinline__ void sha1_compress(uint32_t s[8], const uint32_t M[16])
{
    uint32_t W[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) W[t] = M[t];
    uint32_t a = s[0], b = s[1], c = s[2], d = s[3], e = s[4];
#pragma unroll
    for (int t = 0; t < 80; ++t) {
        if (t >= 16)
            W[t & 15] = rotl<1>(bitop3<TT_XOR3>(W[(t - 3) & 15], W[(t - 8) & 15], W[(t - 14) & 15]) ^ W[t & 15]);
        uint32_t f, k;
        if (t < 20) { f = bitop3<TT_CH>(b, c, d); k = 0x5a827999u; }
        else if (t < 40) { f = bitop3<TT_XOR3>(b, c, d); k = 0x6ed9eba1u; }
        else if (t < 60) { f = bitop3<TT_MAJ>(b, c, d); k = 0x8f1bbcdcu; }
        else { f = bitop3<TT_XOR3>(b, c, d); k = 0xca62c1d6u; }
        uint32_t T = rotl<5>(a) + f + (e + W[t & 15] + k);
        e = d; d = c; c = rotl<30>(b); b = a; a = T;
    }
    s[0] += a; s[1] += b; s[2] += c; s[3] += d; s[4] += e;
}

// ---------------------------------------------------------------------------------------
// SM3 (GB/T 32905-2016 Sec. 4.1-4.4, 5.3.2, 5.3.3)
// ---------------------------------------------------------------------------------------

__device__ __forceinline__ void sm3_init(uint32_t s[8])
{
    s[0] = 0x7380166fu; s[1] = 0x4914b2b9u; s[2] = 0x172442d7u; s[3] = 0xda8a0600u;
    s[4] = 0xa96f30bcu; s[5] = 0x163138aau; s[6] = 0xe38dee4du; s[7] = 0xb0fb0e4eu;
}

__device__ __forceinline__ uint32_t sm3_p0(uint32_t x) { return bitop3<TT_XOR3>(x, rotl<9>(x), rotl<17>(x)); }

// T_j rotated left by j mod 32, folded at compile time.
constexpr uint32_t sm3_tj(int j)
{
    uint32_t t = j < 16 ? 0x79cc4519u : 0x7a879d8au;
    int s = j & 31;
    return s ? ((t << s) | (t >> (32 - s))) : t;
}

// Expansion W_16..W_67 is produced four rounds ahead of use (round j needs W_{j+4} for
// W'_j = W_j ^ W_{j+4}); the xor of W'_j is folded into the TT1 sum with v_xad_u32.
__device__ __forceinline__ void sm3_compress(uint32_t s[8], const uint32_t M[16])
{
    uint32_t W[68];
#pragma unroll
    for (int j = 0; j < 16; ++j) W[j] = M[j];
    uint32_t A = s[0], B = s[1], C = s[2], D = s[3], E = s[4], F = s[5], G = s[6], H = s[7];
#pragma unroll
    for (int j = 0; j < 64; ++j) {
        if (j + 4 >= 16) {
            const int i = j + 4;
            uint32_t x = bitop3<TT_XOR3>(W[i - 16], W[i - 9], rotl<15>(W[i - 3]));
            W[i] = bitop3<TT_XOR3>(bitop3<TT_XOR3>(x, rotl<15>(x), rotl<23>(x)), rotl<7>(W[i - 13]), W[i - 6]);
        }
        uint32_t a12 = rotl<12>(A);
        uint32_t ss1 = rotl<7>(a12 + E + sm3_tj(j));
        uint32_t ff, gg;
        if (j < 16) { ff = bitop3<TT_XOR3>(A, B, C); gg = bitop3<TT_XOR3>(E, F, G); }
        else { ff = bitop3<TT_MAJ>(A, B, C); gg = bitop3<TT_CH>(E, F, G); }
        uint32_t tt1 = ((ss1 ^ a12) + D) + ((W[j] ^ W[j + 4]) + ff);
        uint32_t tt2 = gg + H + ss1 + W[j];
        D = C; C = rotl<9>(B); B = A; A = tt1;
        H = G; G = rotl<19>(F); F = E; E = sm3_p0(tt2);
    }
    s[0] ^= A; s[1] ^= B; s[2] ^= C; s[3] ^= D; s[4] ^= E; s[5] ^= F; s[6] ^= G; s[7] ^= H;
}

// ---------------------------------------------------------------------------------------
// Generic dispatch helpers
// ---------------------------------------------------------------------------------------

template <int A> __device__ __forceinline__ void init_state(uint32_t s[8])
{
    if constexpr (A == MD5) md5_init(s);
    else if constexpr (A == SHA1) sha1_init(s);
    else sm3_init(s);
}

template <int A> __device__ __forceinline__ void compress(uint32_t s[8], const uint32_t w[16])
{
    if constexpr (A == MD5) md5_compress(s, w);
    else if constexpr (A == SHA1) sha1_compress(s, w);
    else sm3_compress(s, w);
}

// ---------------------------------------------------------------------------------------
// Message reading
// ---------------------------------------------------------------------------------------

// A lane's view of its message: the dword holding the first byte, the byte offset r of
// that byte inside it, the byte length and the v_perm selector for the algorithm's word
// order.  Only dwords that hold at least one message byte are ever read, so no access
// leaves the pages the message occupies.
struct Msg {
    const HB_GLOBAL uint32_t *p;
    uint64_t len;
    uint64_t bits;   // value of the padding's length field: 8 x (all bytes hashed so far + len)
    uint32_t r;
    uint32_t sel;
};

template <int A> __device__ __forceinline__ Msg make_msg(const uint8_t *base, uint64_t len)
{
    uintptr_t a = reinterpret_cast<uintptr_t>(base);
    Msg m;
    m.p = reinterpret_cast<const HB_GLOBAL uint32_t *>(a & ~uintptr_t(3));
    m.r = uint32_t(a & 3u);
    m.len = len;
    m.bits = len << 3;
    m.sel = Traits<A>::kBE ? sel_be(m.r) : sel_le(m.r);
    return m;
}

// The 17 dwords covering whole block blk (the 17th holds message bytes only when r != 0;
// for r == 0 dword 15 is re-read in its place, so no read leaves the message's dwords).
__device__ __forceinline__ void load_raw_block(const Msg &m, uint64_t blk, uint32_t raw[17])
{
    const HB_GLOBAL uint32_t *q = m.p + blk * 16u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        u32x4 v = *reinterpret_cast<const HB_GLOBAL u32x4_a4 *>(q + 4 * k);
        raw[4 * k + 0] = v.x; raw[4 * k + 1] = v.y; raw[4 * k + 2] = v.z; raw[4 * k + 3] = v.w;
    }
    raw[16] = q[m.r ? 16 : 15];
}

// Block blk lies wholly inside the message: 16 words from 17 dwords (the 17th holds
// message bytes only when r != 0; for r == 0 dword 15 is re-read in its place).
__device__ __forceinline__ void load_full_block(const Msg &m, uint64_t blk, uint32_t w[16])
{
    const HB_GLOBAL uint32_t *q = m.p + blk * 16u;
    uint32_t raw[17];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        u32x4 v = *reinterpret_cast<const HB_GLOBAL u32x4_a4 *>(q + 4 * k);
        raw[4 * k + 0] = v.x; raw[4 * k + 1] = v.y; raw[4 * k + 2] = v.z; raw[4 * k + 3] = v.w;
    }
    raw[16] = q[m.r ? 16 : 15];
#pragma unroll
    for (int i = 0; i < 16; ++i) w[i] = perm(raw[i + 1], raw[i], m.sel);
}

// Blocks blk and blk + 1, both wholly inside the message, from one burst of 33 dwords:
// the two halves of each 128-byte L2 line are read together rather than one block apart,
// so the line is not evicted and fetched again between them.  `aligned` (wave-uniform)
// means every lane's message starts on a dword, so little-endian words need no realignment.
template <bool BE>
__device__ __forceinline__ void load_full_pair(const Msg &m, uint64_t blk, bool aligned, uint32_t w0[16],
                                               uint32_t w1[16])
{
    const HB_GLOBAL uint32_t *q = m.p + blk * 16u;
    uint32_t raw[33];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        u32x4 v = *reinterpret_cast<const HB_GLOBAL u32x4_a4 *>(q + 4 * k);
        raw[4 * k + 0] = v.x; raw[4 * k + 1] = v.y; raw[4 * k + 2] = v.z; raw[4 * k + 3] = v.w;
    }
    if (!BE && aligned) {
#pragma unroll
        for (int i = 0; i < 16; ++i) { w0[i] = raw[i]; w1[i] = raw[16 + i]; }
        return;
    }
    raw[32] = q[m.r ? 32 : 31];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        w0[i] = perm(raw[i + 1], raw[i], m.sel);
        w1[i] = perm(raw[i + 17], raw[i + 16], m.sel);
    }
}

// Blocks blk .. blk + 3, all wholly inside the message, from one burst of 65 dwords (two
// whole 128-byte L2 lines per lane).
template <bool BE>
__device__ __forceinline__ void load_full_quad(const Msg &m, uint64_t blk, bool aligned, uint32_t w[4][16])
{
    const HB_GLOBAL uint32_t *q = m.p + blk * 16u;
    uint32_t raw[65];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        u32x4 v = *reinterpret_cast<const HB_GLOBAL u32x4_a4 *>(q + 4 * k);
        raw[4 * k + 0] = v.x; raw[4 * k + 1] = v.y; raw[4 * k + 2] = v.z; raw[4 * k + 3] = v.w;
    }
    if (!BE && aligned) {
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int i = 0; i < 16; ++i) w[b][i] = raw[16 * b + i];
        return;
    }
    raw[64] = q[m.r ? 64 : 63];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int i = 0; i < 16; ++i) w[b][i] = perm(raw[16 * b + i + 1], raw[16 * b + i], m.sel);
}

// Any block of the padded message, including the tail block (message bytes, 0x80,
// zeros), the length-only block and, when `last`, the 64-bit bit length in words 14-15
// (low word first for MD5, high word first for SHA-1 / SM3).
template <bool BE>
__device__ __forceinline__ void load_any_block(const Msg &m, uint64_t blk, bool last, uint32_t w[16])
{
    const HB_GLOBAL uint32_t *q = m.p + blk * 16u;
    const int64_t rem = int64_t(m.len) - int64_t(blk * 64u);     // message bytes from block start
    const int32_t v = rem <= 0 ? 0 : (rem >= 64 ? 64 : int32_t(rem)); // valid bytes in block
    const int32_t mk = (rem >= 0 && rem < 64) ? int32_t(rem) : -1;  // position of the 0x80 byte
    const int32_t lim = v > 0 ? v + int32_t(m.r) : 0;               // dword k is read iff 4k < lim
    uint32_t raw[17];
#pragma unroll
    for (int k = 0; k < 17; ++k) raw[k] = (4 * k < lim) ? q[k] : 0u;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        uint32_t x = perm(raw[i + 1], raw[i], m.sel);
        const int32_t d = v - 4 * i;  // message bytes in word i (clamped below)
        uint32_t keep;
        if (BE) keep = d >= 4 ? 0xffffffffu : (d <= 0 ? 0u : (0xffffffffu << (32 - 8 * d)));
        else keep = d >= 4 ? 0xffffffffu : (d <= 0 ? 0u : (0xffffffffu >> (32 - 8 * d)));
        uint32_t mark = 0u;
        if ((mk >> 2) == i) mark = BE ? (0x80u << (24 - 8 * (mk & 3))) : (0x80u << (8 * (mk & 3)));
        w[i] = (x & keep) | mark;
    }
    if (last) {
        const uint64_t bits = m.bits;
        const uint32_t lo = uint32_t(bits), hi = uint32_t(bits >> 32);
        w[14] = BE ? hi : lo;
        w[15] = BE ? lo : hi;
    }
}

// Whole blocks read per burst by default: MD5 does the least work per byte, so it reads
// four (two whole 128-byte L2 lines per lane); SHA-1 and SM3 two (one line).
template <int A> constexpr int kDefaultBurst = A == MD5 ? 4 : 2;

// Absorb the piece m into the chaining value s: its floor(L / 64) whole blocks are read
// directly, up to BURST (1, 2 or 4) per burst; with PAD the remaining one or two blocks of
// nb = floor((L + 8) / 64) + 1 -- tail bytes, 0x80, zeros and the length field m.bits --
// are assembled in registers.  When every lane of a wave has the same length the loop and
// its branch are wave-uniform.
template <int A, bool PAD, int BURST = kDefaultBurst<A>>
__device__ __forceinline__ void absorb(const Msg &m, uint32_t s[8])
{
    static_assert(BURST == 1 || BURST == 2 || BURST == 4, "blocks per burst");
    const uint64_t nfast = m.len / 64u;
    const uint64_t nb = PAD ? (m.len + 8u) / 64u + 1u : nfast;
    // Bursts stop at nb - 2 blocks: every lane's first nb - 2 blocks are whole (nfast is
    // nb - 1 or nb - 2), so lanes of equal nb -- a bucketed wave -- run the burst loops the
    // same number of times and part only for the last two blocks.  nfast and nb are
    // per-lane values; the loops below are per-lane loops that agree when those do.
    uint64_t nburst = PAD ? (nb >= 2u ? nb - 2u : 0u) : nfast;
    if (PAD) {
        // all active lanes with the same nfast (a fixed-length batch): bursts run to it
        const int lead = __ffsll(static_cast<unsigned long long>(__ballot(1))) - 1;
        const unsigned long long nf_lead = __shfl(static_cast<unsigned long long>(nfast), lead);
        if (__all(nfast == nf_lead)) nburst = nfast;
    }
    uint64_t blk = 0;
    // bursts of whole blocks (four, then two), so both halves of each 128-byte line are read
    // before it can be evicted; little-endian words of dword-aligned messages (every lane of
    // the wave) need no realignment
    constexpr bool kBE = Traits<A>::kBE;
    const bool aligned = !kBE && __ballot(m.r != 0) == 0;
    if constexpr (BURST >= 4) {
        for (; blk + 4 <= nburst; blk += 4) {
            uint32_t w[4][16];
            load_full_quad<kBE>(m, blk, aligned, w);
            compress<A>(s, w[0]);
            compress<A>(s, w[1]);
            compress<A>(s, w[2]);
            compress<A>(s, w[3]);
        }
    }
    if constexpr (BURST >= 2) {
        for (; blk + 2 <= nburst; blk += 2) {
            uint32_t w0[16], w1[16];
            load_full_pair<kBE>(m, blk, aligned, w0, w1);
            compress<A>(s, w0);
            compress<A>(s, w1);
        }
    }
    for (; blk < nb; ++blk) {
        uint32_t w[16];
        if (blk < nfast) load_full_block(m, blk, w);
        else load_any_block<Traits<A>::kBE>(m, blk, blk + 1 == nb, w);
        compress<A>(s, w);
    }
}

// Digest state of one whole message: the initial value, then every block including the
// padding.
template <int A, int BURST = kDefaultBurst<A>>
__device__ __forceinline__ void hash_message(const uint8_t *base, uint64_t len, uint32_t s[8])
{
    const Msg m = make_msg<A>(base, len);
    init_state<A>(s);
    absorb<A, true, BURST>(m, s);
}

// As hash_message, with the next whole block's loads issued before the current block is
// compressed, so a lane's memory latency is hidden behind its own compression even when
// few waves share the SIMD.  Two raw buffers, loop unrolled by two: a single loop-carried
// buffer makes the compiler land the next block in fresh registers and copy them over,
// waiting for the loads before the compression instead of after it.  The prefetch is
// unconditional (the last whole block is re-read at the end): loads under a branch make
// the wait before the next block count them as possibly absent and wait for them too.
// Costs 34 VGPRs.
template <int A>
__device__ __forceinline__ void hash_message_prefetch(const uint8_t *base, uint64_t len, uint32_t s[8])
{
    const Msg m = make_msg<A>(base, len);
    const uint64_t nb = (len + 8u) / 64u + 1u;
    const uint64_t nfast = len / 64u;
    init_state<A>(s);
    uint32_t ra[17], rb[17];
    uint64_t blk = 0;
    if (nfast > 0) load_raw_block(m, 0, ra);
    while (blk < nfast) {
        uint32_t w[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) w[i] = perm(ra[i + 1], ra[i], m.sel);
        load_raw_block(m, blk + 1 < nfast ? blk + 1 : blk, rb);
        compress<A>(s, w);
        if (++blk >= nfast) break;
#pragma unroll
        for (int i = 0; i < 16; ++i) w[i] = perm(rb[i + 1], rb[i], m.sel);
        load_raw_block(m, blk + 1 < nfast ? blk + 1 : blk, ra);
        compress<A>(s, w);
        ++blk;
    }
    for (; blk < nb; ++blk) {
        uint32_t w[16];
        load_any_block<Traits<A>::kBE>(m, blk, blk + 1 == nb, w);
        compress<A>(s, w);
    }
}

// Canonical digest bytes: MD5 registers as stored (little-endian), SHA-1 / SM3 words
// byte-reversed.  Slot bytes past the digest (up to `stride`) are written as zero.
template <int A>
__device__ __forceinline__ void store_digest(uint8_t *out, const uint32_t s[8], uint32_t stride)
{
    HB_GLOBAL uint32_t *o = reinterpret_cast<HB_GLOBAL uint32_t *>(reinterpret_cast<uintptr_t>(out));
#pragma unroll
    for (int q = 0; q < Traits<A>::kWords; ++q) o[q] = Traits<A>::kBE ? bswap32(s[q]) : s[q];
    for (uint32_t q = Traits<A>::kWords; q < stride / 4u; ++q) o[q] = 0u;
}

}  // namespace hb
