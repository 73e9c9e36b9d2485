// hb_long.hpp -- long Merkle-Damgard chains with the per-block work that does not depend
// on the chaining value moved off the chain.
//
// A message's blocks must be compressed one after another, so a long message is a
// critical path no amount of parallelism shortens.  What can leave the chain is every
// operation that depends only on the block's words: the SHA-1 and SM3 message schedules
// (FIPS 180-4 Sec. 6.1.2 step 1; GB/T 32905 Sec. 5.3.2), and the additions of round
// constants to schedule words that feed a sum anyway.  One lane per (message, block)
// computes those words into scratch memory ahead of time; the chain then runs the rounds
// only, reading them back:
//   MD5   XT[i] = X[k(i)] + T[i]          64 words  -> 4 ops per step instead of 5
//   SHA-1 WK[t] = W[t] + K(t)             80 words  -> no schedule on the chain
//   SM3   W'[j], W[j] for j = 0..63      128 words  -> no expansion, W' sum folded
#pragma once

#include "hb_device.hpp"

namespace hb {

constexpr int kSchedWords = 128;  // scratch words per block (the largest of the three)

template <int A> struct SchedWords;
template <> struct SchedWords<MD5> { static constexpr int kN = 64; };
template <> struct SchedWords<SHA1> { static constexpr int kN = 80; };
template <> struct SchedWords<SM3> { static constexpr int kN = 128; };

// ---------------------------------------------------------------------------------------
// Schedule computation for one block (one lane per block)
// ---------------------------------------------------------------------------------------

__device__ __forceinline__ void md5_sched(const uint32_t X[16], uint32_t out[64])
{
    constexpr const uint32_t *T = kMd5T;
#pragma unroll
    for (int i = 0; i < 64; ++i) {
        const int j = i & 15;
        const int k = i < 16 ? j : (i < 32 ? (1 + 5 * j) & 15 : (i < 48 ? (5 + 3 * j) & 15 : (7 * j) & 15));
        out[i] = X[k] + T[i];
    }
}

__device__ __forceinline__ void sha1_sched(const uint32_t M[16], uint32_t out[80])
{
    uint32_t W[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) W[t] = M[t];
#pragma unroll
    for (int t = 0; t < 80; ++t) {
        if (t >= 16)
            W[t & 15] = rotl<1>(bitop3<TT_XOR3>(W[(t - 3) & 15], W[(t - 8) & 15], W[(t - 14) & 15]) ^ W[t & 15]);
        const uint32_t k = t < 20 ? 0x5a827999u : (t < 40 ? 0x6ed9eba1u : (t < 60 ? 0x8f1bbcdcu : 0xca62c1d6u));
        out[t] = W[t & 15] + k;
    }
}

// out[0..63] = W'_j, out[64..127] = W_j
__device__ __forceinline__ void sm3_sched(const uint32_t M[16], uint32_t out[128])
{
    uint32_t W[68];
#pragma unroll
    for (int j = 0; j < 16; ++j) W[j] = M[j];
#pragma unroll
    for (int i = 16; i < 68; ++i) {
        uint32_t x = bitop3<TT_XOR3>(W[i - 16], W[i - 9], rotl<15>(W[i - 3]));
        W[i] = bitop3<TT_XOR3>(bitop3<TT_XOR3>(x, rotl<15>(x), rotl<23>(x)), rotl<7>(W[i - 13]), W[i - 6]);
    }
#pragma unroll
    for (int j = 0; j < 64; ++j) {
        out[j] = W[j] ^ W[j + 4];
        out[64 + j] = W[j];
    }
}

// ---------------------------------------------------------------------------------------
// Rounds only, from precomputed words
// ---------------------------------------------------------------------------------------

// (a ^ b) + c as one v_xad_u32 (the compiler's own pattern match is not reliable once the
// surrounding sums are re-associated).
__device__ __forceinline__ uint32_t xad(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_xad_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ __forceinline__ void md5_rounds(uint32_t s[8], const uint32_t XT[64])
{
    uint32_t a = s[0], b = s[1], c = s[2], d = s[3];
#define HB_MD5_RSTEP(TTF, sh, i)                                  \
    {                                                             \
        uint32_t t = a + bitop3<TTF>(b, c, d) + XT[i];            \
        a = d; d = c; c = b;                                      \
        b = b + rotl<sh>(t);                                      \
    }
#pragma unroll
    for (int j = 0; j < 16; j += 4) {
        HB_MD5_RSTEP(TT_CH, 7, j + 0) HB_MD5_RSTEP(TT_CH, 12, j + 1)
        HB_MD5_RSTEP(TT_CH, 17, j + 2) HB_MD5_RSTEP(TT_CH, 22, j + 3)
    }
#pragma unroll
    for (int j = 16; j < 32; j += 4) {
        HB_MD5_RSTEP(TT_MD5_G, 5, j + 0) HB_MD5_RSTEP(TT_MD5_G, 9, j + 1)
        HB_MD5_RSTEP(TT_MD5_G, 14, j + 2) HB_MD5_RSTEP(TT_MD5_G, 20, j + 3)
    }
#pragma unroll
    for (int j = 32; j < 48; j += 4) {
        HB_MD5_RSTEP(TT_XOR3, 4, j + 0) HB_MD5_RSTEP(TT_XOR3, 11, j + 1)
        HB_MD5_RSTEP(TT_XOR3, 16, j + 2) HB_MD5_RSTEP(TT_XOR3, 23, j + 3)
    }
#pragma unroll
    for (int j = 48; j < 64; j += 4) {
        HB_MD5_RSTEP(TT_MD5_I, 6, j + 0) HB_MD5_RSTEP(TT_MD5_I, 10, j + 1)
        HB_MD5_RSTEP(TT_MD5_I, 15, j + 2) HB_MD5_RSTEP(TT_MD5_I, 21, j + 3)
    }
#undef HB_MD5_RSTEP
    s[0] += a; s[1] += b; s[2] += c; s[3] += d;
}

__device__ __forceinline__ void sha1_rounds(uint32_t s[8], const uint32_t WK[80])
{
    uint32_t a = s[0], b = s[1], c = s[2], d = s[3], e = s[4];
#pragma unroll
    for (int t = 0; t < 80; ++t) {
        uint32_t f;
        if (t < 20) f = bitop3<TT_CH>(b, c, d);
        else if (t < 40) f = bitop3<TT_XOR3>(b, c, d);
        else if (t < 60) f = bitop3<TT_MAJ>(b, c, d);
        else f = bitop3<TT_XOR3>(b, c, d);
        uint32_t T = rotl<5>(a) + f + (e + WK[t]);
        e = d; d = c; c = rotl<30>(b); b = a; a = T;
    }
    s[0] += a; s[1] += b; s[2] += c; s[3] += d; s[4] += e;
}

__device__ __forceinline__ void sm3_rounds(uint32_t s[8], const uint32_t WW[128])
{
    uint32_t A = s[0], B = s[1], C = s[2], D = s[3], E = s[4], F = s[5], G = s[6], H = s[7];
#pragma unroll
    for (int j = 0; j < 64; ++j) {
        uint32_t a12 = rotl<12>(A);
        uint32_t ss1 = rotl<7>(a12 + E + sm3_tj(j));
        uint32_t ff, gg;
        if (j < 16) { ff = bitop3<TT_XOR3>(A, B, C); gg = bitop3<TT_XOR3>(E, F, G); }
        else { ff = bitop3<TT_MAJ>(A, B, C); gg = bitop3<TT_CH>(E, F, G); }
        uint32_t tt1 = xad(ss1, a12, D + WW[j] + ff);
        uint32_t tt2 = gg + H + ss1 + WW[64 + j];
        D = C; C = rotl<9>(B); B = A; A = tt1;
        H = G; G = rotl<19>(F); F = E; E = sm3_p0(tt2);
    }
    s[0] ^= A; s[1] ^= B; s[2] ^= C; s[3] ^= D; s[4] ^= E; s[5] ^= F; s[6] ^= G; s[7] ^= H;
}

template <int A> __device__ __forceinline__ void sched_block(const uint32_t w[16], uint32_t *out)
{
    if constexpr (A == MD5) md5_sched(w, out);
    else if constexpr (A == SHA1) sha1_sched(w, out);
    else sm3_sched(w, out);
}

template <int A> __device__ __forceinline__ void rounds(uint32_t s[8], const uint32_t *ww)
{
    if constexpr (A == MD5) md5_rounds(s, ww);
    else if constexpr (A == SHA1) sha1_rounds(s, ww);
    else sm3_rounds(s, ww);
}

// Scratch layout, wave-interleaved so each load instruction of a wave reads one
// contiguous KiB: a long-chain wave owns a region of (its longest message's block count)
// "wave-blocks"; in it, word group k (4 words) of block b of lane l sits at words
// ((b * kGroups + k) * 64 + l) * 4.
constexpr int kGroups = kSchedWords / 4;
constexpr uint64_t kWaveBlockWords = uint64_t(kGroups) * 64 * 4;  // 32 KiB

__device__ __forceinline__ uint64_t sched_at(uint64_t b, int k, uint32_t lane)
{
    return ((b * kGroups + uint64_t(k)) * 64u + lane) * 4u;
}

// Load block b's precomputed words (kN of them) of lane `lane` from wave region wr.
template <int A> __device__ __forceinline__ void load_sched(const uint32_t *wr, uint64_t b, uint32_t lane, uint32_t *ww)
{
    const HB_GLOBAL uint32_t *q = reinterpret_cast<const HB_GLOBAL uint32_t *>(reinterpret_cast<uintptr_t>(wr));
#pragma unroll
    for (int k = 0; k < SchedWords<A>::kN / 4; ++k) {
        u32x4 v = *reinterpret_cast<const HB_GLOBAL u32x4 *>(q + sched_at(b, k, lane));
        ww[4 * k + 0] = v.x; ww[4 * k + 1] = v.y; ww[4 * k + 2] = v.z; ww[4 * k + 3] = v.w;
    }
}

// Store block b's words for lane `lane` into wave region wr.
template <int A> __device__ __forceinline__ void store_sched(uint32_t *wr, uint64_t b, uint32_t lane, const uint32_t *ww)
{
    HB_GLOBAL uint32_t *q = reinterpret_cast<HB_GLOBAL uint32_t *>(reinterpret_cast<uintptr_t>(wr));
#pragma unroll
    for (int k = 0; k < SchedWords<A>::kN / 4; ++k)
        *reinterpret_cast<HB_GLOBAL u32x4 *>(q + sched_at(b, k, lane)) =
            u32x4{ww[4 * k + 0], ww[4 * k + 1], ww[4 * k + 2], ww[4 * k + 3]};
}

// The chain of a message of nb blocks whose words are in wave region wr, lane `lane`:
// rounds only, the next block's words loaded while the current block is compressed (two
// buffers, loop unrolled by two so no copies are needed; every load unconditional so the
// compiler's waits count them exactly).
template <int A>
__device__ __forceinline__ void chain_from_sched(const uint32_t *wr, uint32_t lane, uint64_t nb, uint32_t s[8])
{
    constexpr int N = SchedWords<A>::kN;
    uint32_t w0[N], w1[N];
    init_state<A>(s);
    load_sched<A>(wr, 0, lane, w0);
    uint64_t blk = 0;
    for (; blk + 2 <= nb; blk += 2) {
        load_sched<A>(wr, blk + 1, lane, w1);
        rounds<A>(s, w0);
        // unconditional (the last block is re-read at the end): a load under a branch
        // makes the wait before rounds(w1) count it as possibly absent and wait for it too
        load_sched<A>(wr, blk + 2 < nb ? blk + 2 : blk + 1, lane, w0);
        rounds<A>(s, w1);
    }
    if (blk < nb) rounds<A>(s, w0);
}

}  // namespace hb
