// hb_cpu.cpp -- host-core share of a CPU + GPU split (the duty ratio of Sec. V-D, Eq. 1-3).
//
// The paper splits a batch between CPU cores and the GPU and picks the CPU fraction x that
// balances T_cpu = N P_cpu x / N_core against the GPU's compute, allocation and copy time.
// This file is the CPU side: MD5 (RFC 1321), SHA-1 (FIPS 180-4) and SM3 (GB/T 32905)
// written for a host core -- whole blocks compressed straight from the message, only the
// last one or two padded blocks built in a small buffer -- and a thread pool that spreads
// a range of messages over host threads.  Digests use the GPU path's layout (canonical
// bytes, slot stride, zero fill), so the two halves of a split batch land in one buffer.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

#include "../../include/hb.h"
#include "hb_internal.hpp"
#include "hb_md5_table.hpp"

namespace hb {
namespace {

inline uint32_t rol(uint32_t x, int r) { return r == 0 ? x : (x << r) | (x >> (32 - r)); }
inline uint32_t get_le(const uint8_t *p) { return uint32_t(p[0]) | uint32_t(p[1]) << 8 | uint32_t(p[2]) << 16 | uint32_t(p[3]) << 24; }
inline uint32_t get_be(const uint8_t *p) { return uint32_t(p[0]) << 24 | uint32_t(p[1]) << 16 | uint32_t(p[2]) << 8 | uint32_t(p[3]); }

// ---- MD5, RFC 1321 Sec. 3.4: four rounds of sixteen steps -------------------------------
struct Md5 {
    static constexpr int kWords = 4;
    static constexpr bool kBigEndianLength = false;
    uint32_t h[4] = {0x67452301u, 0xefcdab89u, 0x98badcfeu, 0x10325476u};
    void block(const uint8_t *p)
    {
        const uint32_t *T = kMd5T;
        static const int S[4][4] = {{7, 12, 17, 22}, {5, 9, 14, 20}, {4, 11, 16, 23}, {6, 10, 15, 21}};
        uint32_t x[16];
        for (int i = 0; i < 16; ++i) x[i] = get_le(p + 4 * i);
        uint32_t a = h[0], b = h[1], c = h[2], d = h[3];
        for (int i = 0; i < 64; ++i) {
            const int r = i >> 4;
            uint32_t f;
            int k;
            if (r == 0) { f = (b & c) | (~b & d); k = i; }
            else if (r == 1) { f = (b & d) | (c & ~d); k = (5 * i + 1) & 15; }
            else if (r == 2) { f = b ^ c ^ d; k = (3 * i + 5) & 15; }
            else { f = c ^ (b | ~d); k = (7 * i) & 15; }
            const uint32_t t = d;
            d = c;
            c = b;
            b = b + rol(a + f + x[k] + T[i], S[r][i & 3]);
            a = t;
        }
        h[0] += a; h[1] += b; h[2] += c; h[3] += d;
    }
    void out(uint8_t *o) const
    {
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) o[4 * i + j] = uint8_t(h[i] >> (8 * j));
    }
};

// ---- SHA-1, FIPS 180-4 Sec. 6.1.2 ------------------------------------------------------
struct Sha1 {
    static constexpr int kWords = 5;
    static constexpr bool kBigEndianLength = true;
    uint32_t h[5] = {0x67452301u, 0xefcdab89u, 0x98badcfeu, 0x10325476u, 0xc3d2e1f0u};
    void block(const uint8_t *p)
    {
        uint32_t w[80];
        for (int t = 0; t < 16; ++t) w[t] = get_be(p + 4 * t);
        for (int t = 16; t < 80; ++t) w[t] = rol(w[t - 3] ^ w[t - 8] ^ w[t - 14] ^ w[t - 16], 1);
        uint32_t a = h[0], b = h[1], c = h[2], d = h[3], e = h[4];
        for (int t = 0; t < 80; ++t) {
            uint32_t f, k;
            if (t < 20) { f = (b & c) ^ (~b & d); k = 0x5a827999u; }
            else if (t < 40) { f = b ^ c ^ d; k = 0x6ed9eba1u; }
            else if (t < 60) { f = (b & c) ^ (b & d) ^ (c & d); k = 0x8f1bbcdcu; }
            else { f = b ^ c ^ d; k = 0xca62c1d6u; }
            const uint32_t tmp = rol(a, 5) + f + e + k + w[t];
            e = d; d = c; c = rol(b, 30); b = a; a = tmp;
        }
        h[0] += a; h[1] += b; h[2] += c; h[3] += d; h[4] += e;
    }
    void out(uint8_t *o) const
    {
        for (int i = 0; i < 5; ++i)
            for (int j = 0; j < 4; ++j) o[4 * i + j] = uint8_t(h[i] >> (24 - 8 * j));
    }
};

// ---- SM3, GB/T 32905-2016 Sec. 5.3 -----------------------------------------------------
struct Sm3 {
    static constexpr int kWords = 8;
    static constexpr bool kBigEndianLength = true;
    uint32_t h[8] = {0x7380166fu, 0x4914b2b9u, 0x172442d7u, 0xda8a0600u,
                     0xa96f30bcu, 0x163138aau, 0xe38dee4du, 0xb0fb0e4eu};
    static uint32_t p0(uint32_t x) { return x ^ rol(x, 9) ^ rol(x, 17); }
    static uint32_t p1(uint32_t x) { return x ^ rol(x, 15) ^ rol(x, 23); }
    void block(const uint8_t *p)
    {
        uint32_t w[68], w1[64];
        for (int j = 0; j < 16; ++j) w[j] = get_be(p + 4 * j);
        for (int j = 16; j < 68; ++j)
            w[j] = p1(w[j - 16] ^ w[j - 9] ^ rol(w[j - 3], 15)) ^ rol(w[j - 13], 7) ^ w[j - 6];
        for (int j = 0; j < 64; ++j) w1[j] = w[j] ^ w[j + 4];
        uint32_t A = h[0], B = h[1], C = h[2], D = h[3], E = h[4], F = h[5], G = h[6], H = h[7];
        for (int j = 0; j < 64; ++j) {
            const uint32_t tj = j < 16 ? 0x79cc4519u : 0x7a879d8au;
            const uint32_t ss1 = rol(rol(A, 12) + E + rol(tj, j % 32), 7);
            const uint32_t ss2 = ss1 ^ rol(A, 12);
            const uint32_t ff = j < 16 ? (A ^ B ^ C) : ((A & B) | (A & C) | (B & C));
            const uint32_t gg = j < 16 ? (E ^ F ^ G) : ((E & F) | (~E & G));
            const uint32_t tt1 = ff + D + ss2 + w1[j];
            const uint32_t tt2 = gg + H + ss1 + w[j];
            D = C; C = rol(B, 9); B = A; A = tt1;
            H = G; G = rol(F, 19); F = E; E = p0(tt2);
        }
        h[0] ^= A; h[1] ^= B; h[2] ^= C; h[3] ^= D; h[4] ^= E; h[5] ^= F; h[6] ^= G; h[7] ^= H;
    }
    void out(uint8_t *o) const
    {
        for (int i = 0; i < 8; ++i)
            for (int j = 0; j < 4; ++j) o[4 * i + j] = uint8_t(h[i] >> (24 - 8 * j));
    }
};

// Whole blocks straight from the message; the tail, the 0x80 byte, zeros and the 64-bit
// bit length (little-endian for MD5, big-endian otherwise) in a two-block buffer.
template <class H> void digest_one(const uint8_t *m, uint64_t len, uint8_t *out, uint32_t stride)
{
    H st;
    const uint64_t whole = len / 64u;
    for (uint64_t b = 0; b < whole; ++b) st.block(m + 64u * b);
    uint8_t tail[128] = {};
    const uint32_t rem = uint32_t(len - 64u * whole);
    if (rem) std::memcpy(tail, m + 64u * whole, rem);
    tail[rem] = 0x80;
    const uint32_t nt = rem + 9 <= 64 ? 64u : 128u;
    const uint64_t bits = len * 8u;
    for (int j = 0; j < 8; ++j)
        tail[nt - 8 + j] = uint8_t(H::kBigEndianLength ? bits >> (56 - 8 * j) : bits >> (8 * j));
    st.block(tail);
    if (nt == 128) st.block(tail + 64);
    st.out(out);
    for (uint32_t q = 4u * H::kWords; q < stride; ++q) out[q] = 0;
}

void digest_any(int algo, const uint8_t *m, uint64_t len, uint8_t *out, uint32_t stride)
{
    switch (algo) {
    case 0: digest_one<Md5>(m, len, out, stride); break;
    case 1: digest_one<Sha1>(m, len, out, stride); break;
    case 2: digest_one<Sm3>(m, len, out, stride); break;
    default: std::memset(out, 0, stride);  // unknown id: all-zero slot, as on the GPU
    }
}

}  // namespace

// Hash messages [i0, i1) on `threads` host threads (0: all hardware threads); message i's
// digest goes to out + (i - i0) * stride.  Threads take chunks of messages from a shared
// counter, so a few long messages do not leave the others idle.
void cpu_hash_range(const uint8_t *algos, int algo, const uint8_t *msgs, const uint64_t *offs, const uint64_t *lens,
                    uint64_t i0, uint64_t i1, uint8_t *out, uint32_t stride, int threads)
{
    if (i1 <= i0) return;
    if (threads <= 0) threads = int(std::max(1u, std::thread::hardware_concurrency()));
    constexpr uint64_t kChunk = 64;
    std::atomic<uint64_t> next{i0};
    auto work = [&] {
        for (;;) {
            const uint64_t a = next.fetch_add(kChunk);
            if (a >= i1) return;
            const uint64_t b = std::min(i1, a + kChunk);
            for (uint64_t i = a; i < b; ++i)
                digest_any(algos ? int(algos[i]) : algo, msgs + offs[i], lens[i], out + (i - i0) * stride, stride);
        }
    };
    const uint64_t n = i1 - i0;
    const int t = int(std::min<uint64_t>(uint64_t(threads), (n + kChunk - 1) / kChunk));
    std::vector<std::thread> pool;
    for (int k = 1; k < t; ++k) pool.emplace_back(work);
    work();
    for (auto &th : pool) th.join();
}

}  // namespace hb

using namespace hb;

extern "C" int hb_cpu_hash_batch(const uint8_t *algos_host, int algo, const uint8_t *messages_host,
                                 const uint64_t *offsets_host, const uint64_t *lengths_host, uint64_t n,
                                 uint8_t *digests_out_host, int threads)
{
    if (!algos_host && digest_size(algo) == 0) return set_error(HB_EINVAL, "hb_cpu_hash_batch: unknown algorithm id");
    if (n == 0) return HB_OK;
    if (!offsets_host || !lengths_host || !digests_out_host)
        return set_error(HB_EINVAL, "hb_cpu_hash_batch: null host pointer");
    uint64_t any = 0;
    for (uint64_t i = 0; i < n; ++i) any |= lengths_host[i];
    if (any && !messages_host) return set_error(HB_EINVAL, "hb_cpu_hash_batch: null messages");
    const uint32_t stride = algos_host ? 32u : uint32_t(digest_size(algo));
    cpu_hash_range(algos_host, algo, messages_host, offsets_host, lengths_host, 0, n, digests_out_host, stride, threads);
    return HB_OK;
}
