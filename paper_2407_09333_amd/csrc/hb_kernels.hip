// hb_kernels.hip -- plain batch-hashing kernels: one lane per message, in index order.
#include <algorithm>
#include <cstdlib>

#include "hb_device.hpp"
#include "hb_internal.hpp"

namespace hb {

constexpr int kPlainBlock = 256;

// Workgroups are dealt round-robin to the GPU's XCDs (8 on MI355X, each with its own L2);
// renumbering them so that each XCD takes a contiguous run of the grid makes each XCD
// stream through one contiguous region of the input.  Measured on 2^20 x 1 KiB MD5: 205 us
// against 210 us in dispatch order; a load-only stream: 5.7 against 5.4 TB/s.
constexpr uint32_t kXcds = 8;

__device__ __forceinline__ uint32_t xcd_contiguous_block()
{
    const uint32_t b = blockIdx.x, full = gridDim.x & ~(kXcds - 1u);
    if (b >= full) return b;  // the last gridDim % 8 workgroups keep their number
    return (b % kXcds) * (full / kXcds) + b / kXcds;
}

// Lane i hashes message i.  FIXED: message i starts at i * fixed_len and is fixed_len
// bytes long (no metadata reads).  With `filter`, messages whose id differs from A are
// skipped, so one launch per algorithm covers a mixed batch.
template <int A, bool FIXED>
__global__ __launch_bounds__(kPlainBlock) void k_plain(const uint8_t *__restrict__ msgs,
                                                       const uint64_t *__restrict__ offs,
                                                       const uint64_t *__restrict__ lens, uint64_t n,
                                                       uint64_t fixed_len, uint8_t *__restrict__ out,
                                                       uint32_t stride,
                                                       const uint8_t *__restrict__ filter)
{
    const uint64_t i = uint64_t(xcd_contiguous_block()) * kPlainBlock + threadIdx.x;
    if (i >= n) return;
    if (filter) {
        const uint8_t id = filter[i];
        if (id != A) {
            if (A == MD5 && id > SM3) {  // unknown id: an all-zero slot
                HB_GLOBAL uint32_t *o = reinterpret_cast<HB_GLOBAL uint32_t *>(reinterpret_cast<uintptr_t>(out + i * stride));
                for (uint32_t q = 0; q < stride / 4u; ++q) o[q] = 0u;
            }
            return;
        }
    }
    uint64_t off, len;
    if constexpr (FIXED) { off = i * fixed_len; len = fixed_len; }
    else { off = offs[i]; len = lens[i]; }
    uint32_t s[8];
    hash_message<A>(msgs + off, len, s);
    store_digest<A>(out + i * stride, s, stride);
}

// Buffer resource word 3 for raw (unswizzled, unformatted) dword access on gfx9-family
// GPUs, and the cache-policy bit of a non-temporal buffer load.
constexpr int kBufferRsrcWord3 = 0x00020000;
constexpr int kCpolNonTemporal = 2;

// Fixed-length batch with message words staged through LDS (the default for dword-aligned
// fixed-length batches; HB_PLAIN_LDS=0 takes k_plain instead).  Each wave owns 64
// consecutive messages.  Two whole blocks of all 64 go per burst: eight 16-byte loads per
// lane, lane (q, p) of load j taking chunk p ^ q of message 8j + q, so each load instruction
// reads eight whole 128-byte lines; the chunks are written to the wave's LDS slice in that
// order and each lane reads back its own message's 128 bytes, the XOR swizzle putting eight
// consecutive lanes on eight different bank groups.  Messages must start on a dword (msgs
// and msg_len 4-byte aligned); the last one or two blocks and a partial last wave go through
// the per-lane path.  The loads are buffer loads off one wave-uniform base, so they take no
// vector address arithmetic (MD5 issues its compression instructions and almost nothing
// more) and few registers.  Each wave keeps the next burst in flight while it compresses the
// current one.  MD5, whose reads and compression take about as long as each other, streams
// with non-temporal loads (every line is read once, whole, by one instruction) at five waves
// per SIMD, the most the LDS holds (8 KiB per wave); SHA-1 and SM3, bound by their
// compression, use cached loads at five and four.  In interleaved runs on 2^20 x 1 KiB
// against the per-lane kernel: MD5 0.92, SHA-1 0.98, SM3 0.98 of its time.
template <int A>
__global__ __launch_bounds__(kPlainBlock) __attribute__((amdgpu_waves_per_eu(A == MD5 ? 5 : 4))) void k_plain_lds(const uint8_t *__restrict__ msgs, uint64_t n,
                                                           uint64_t len, uint8_t *__restrict__ out)
{
    constexpr bool kStream = A == MD5;  // non-temporal loads
    __shared__ u32x4 slice[kPlainBlock / 64][512];  // per wave: 64 messages x 128 bytes
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64u), lane = threadIdx.x % 64u;
    const uint64_t m0 = (uint64_t(xcd_contiguous_block()) * (kPlainBlock / 64) + wave) * 64u;
    if (m0 >= n) return;
    const uint32_t q = lane / 8u, p = lane % 8u, sw = lane & 7u;
    const uint32_t voff = uint32_t(q * len + (p ^ q) * 16u);  // load j adds 8 j len
    const uint64_t nb = (len + 8u) / 64u + 1u, nfast = len / 64u;
    const uint64_t nburst = m0 + 64u <= n ? nfast / 2u : 0u;  // wave-uniform
    const uint8_t *wbase = msgs + m0 * len;
    u32x4 *mine = slice[wave];
    uint32_t s[8];
    init_state<A>(s);
    // The wave's 64 messages through one buffer resource: base in SGPRs, the lane's 32-bit
    // offset in one VGPR, the burst's and load's offset (k 128 + 8 j len) in an SGPR, so a
    // load costs no vector address arithmetic and the loop keeps no 64-bit addresses.  Its
    // range is the wave's 64 messages, 64 len bytes (< 2^31 for the lengths taken here):
    // the furthest load, burst nburst - 1 of message 63, ends at 63 len + 128 nburst <= 64 len,
    // and a read past the range would return zeros rather than touch other memory.  Only
    // whole waves (m0 + 64 <= n) use it.
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(wbase), 0, int(64u * uint32_t(len)), kBufferRsrcWord3);
    auto load = [&](u32x4 *pre, uint64_t k) {
#pragma unroll
        for (int j = 0; j < 8; ++j)
            pre[j] = __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff, uint32_t(k * 128u + uint64_t(8 * j) * len),
                                                           kStream ? kCpolNonTemporal : 0);
    };
    auto stage = [&](const u32x4 *pre) {
#pragma unroll
        for (int j = 0; j < 8; ++j) mine[j * 64 + lane] = pre[j];
    };
    // The two staged blocks of this lane's message.  MD5 and SHA-1 read both blocks' words
    // from LDS up front, so the second block's reads complete under the first block's
    // compression (16 more registers; SM3, with more state live, reads one block at a time
    // to stay within four waves per SIMD).
    constexpr bool kReadAhead = A != SM3;
    auto words = [&](int h, uint32_t *w) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const u32x4 v = mine[lane * 8u + ((4u * h + i) ^ sw)];
            w[4 * i] = v.x; w[4 * i + 1] = v.y; w[4 * i + 2] = v.z; w[4 * i + 3] = v.w;
        }
        if (Traits<A>::kBE)
#pragma unroll
            for (int i = 0; i < 16; ++i) w[i] = bswap32(w[i]);
    };
    auto burst = [&]() {
        if constexpr (kReadAhead) {
            uint32_t w0[16], w1[16];
            // block 0's reads, then block 1's, both before block 0's compression: the wait
            // for block 0 leaves block 1's reads in flight under it
            words(0, w0);
            __builtin_amdgcn_sched_barrier(0);
            words(1, w1);
            __builtin_amdgcn_sched_barrier(0);
            compress<A>(s, w0);
            compress<A>(s, w1);
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                uint32_t w[16];
                words(h, w);
                compress<A>(s, w);
            }
        }
    };
    // A wave's LDS operations complete in order, so a burst's writes to the slice follow the
    // previous burst's reads of it.
    u32x4 pre[8];
    if (nburst) load(pre, 0);
    for (uint64_t k = 0; k < nburst; ++k) {
        stage(pre);
        if (k + 1 < nburst) load(pre, k + 1);
        burst();
    }
    const uint64_t mi = m0 + lane;
    if (mi >= n) return;
    const Msg m = make_msg<A>(msgs + mi * len, len);
    uint64_t blk = nburst * 2u;
    for (; blk < nfast; ++blk) {
        uint32_t w[16];
        load_full_block(m, blk, w);
        compress<A>(s, w);
    }
    if (len % 64u == 0) {
        // the last block is padding only -- 0x80, zeros, the bit length -- and the same for
        // every message of the batch: wave-uniform words, nothing to read or assemble
        constexpr bool kBE = Traits<A>::kBE;
        uint32_t w[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) w[i] = 0u;
        w[0] = kBE ? 0x80000000u : 0x80u;
        const uint64_t bits = len << 3;
        w[14] = kBE ? uint32_t(bits >> 32) : uint32_t(bits);
        w[15] = kBE ? uint32_t(bits) : uint32_t(bits >> 32);
        compress<A>(s, w);
    } else {
        for (; blk < nb; ++blk) {
            uint32_t w[16];
            load_any_block<Traits<A>::kBE>(m, blk, blk + 1 == nb, w);
            compress<A>(s, w);
        }
    }
    store_digest<A>(out + mi * Traits<A>::kDigest, s, Traits<A>::kDigest);
}

// The paper's workload (Sec. V-A.2): message i is the 9-character decimal text of
// start + i, zero-padded ("000000000" .. "999999999").  The text is produced in registers,
// so a 9-byte message is one padded block: 9 bytes, 0x80, zeros, bit length 72.
template <int A>
__global__ __launch_bounds__(kPlainBlock) void k_digits9(uint64_t start, uint64_t n, uint8_t *__restrict__ out)
{
    const uint64_t i = uint64_t(blockIdx.x) * kPlainBlock + threadIdx.x;
    if (i >= n) return;
    uint32_t v = uint32_t(start + i);  // < 10^9
    uint32_t d[9];
#pragma unroll
    for (int k = 8; k >= 0; --k) {
        const uint32_t q = v / 10u;
        d[k] = 0x30u + (v - q * 10u);
        v = q;
    }
    uint32_t w[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) w[k] = 0u;
    if (Traits<A>::kBE) {
        w[0] = (d[0] << 24) | (d[1] << 16) | (d[2] << 8) | d[3];
        w[1] = (d[4] << 24) | (d[5] << 16) | (d[6] << 8) | d[7];
        w[2] = (d[8] << 24) | 0x00800000u;
        w[15] = 72u;
    } else {
        w[0] = d[0] | (d[1] << 8) | (d[2] << 16) | (d[3] << 24);
        w[1] = d[4] | (d[5] << 8) | (d[6] << 16) | (d[7] << 24);
        w[2] = d[8] | 0x8000u;
        w[14] = 72u;
    }
    uint32_t s[8];
    init_state<A>(s);
    compress<A>(s, w);
    store_digest<A>(out + i * Traits<A>::kDigest, s, Traits<A>::kDigest);
}

// Byte copy between device-accessible buffers (device memory or the device mapping of
// pinned host memory): 16 bytes per lane per step when both ends are 16-byte aligned.
template <bool VEC>
__global__ __launch_bounds__(256) void k_copy(uint8_t *dst, const uint8_t *src, uint64_t n)
{
    const uint64_t t = uint64_t(blockIdx.x) * 256u + threadIdx.x, step = uint64_t(gridDim.x) * 256u;
    uint64_t head = 0;
    if constexpr (VEC) {
        const uint64_t nv = n / 16u;
        for (uint64_t i = t; i < nv; i += step)
            reinterpret_cast<u32x4 *>(dst)[i] = reinterpret_cast<const u32x4 *>(src)[i];
        head = nv * 16u;
    }
    for (uint64_t i = head + t; i < n; i += step) dst[i] = src[i];
}

hipError_t launch_copy(void *dst, const void *src, uint64_t bytes, hipStream_t stream)
{
    if (bytes == 0) return hipSuccess;
    const bool vec = ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15u) == 0;
    const uint64_t units = vec ? (bytes + 15u) / 16u : bytes;
    const unsigned blocks = unsigned(std::min<uint64_t>((units + 255u) / 256u, 2048u));
    if (vec)
        hipLaunchKernelGGL(k_copy<true>, dim3(blocks), dim3(256), 0, stream, static_cast<uint8_t *>(dst),
                           static_cast<const uint8_t *>(src), bytes);
    else
        hipLaunchKernelGGL(k_copy<false>, dim3(blocks), dim3(256), 0, stream, static_cast<uint8_t *>(dst),
                           static_cast<const uint8_t *>(src), bytes);
    return hipGetLastError();
}

hipError_t launch_digits9(int algo, uint64_t start, uint64_t n, uint8_t *out, hipStream_t stream)
{
    const uint64_t blocks = (n + kPlainBlock - 1) / kPlainBlock;
    if (blocks > 0x7fffffffull) return hipErrorInvalidConfiguration;
    const dim3 grid{uint32_t(blocks), 1, 1}, block{kPlainBlock, 1, 1};
    switch (algo) {
    case MD5: hipLaunchKernelGGL(k_digits9<MD5>, grid, block, 0, stream, start, n, out); break;
    case SHA1: hipLaunchKernelGGL(k_digits9<SHA1>, grid, block, 0, stream, start, n, out); break;
    case SM3: hipLaunchKernelGGL(k_digits9<SM3>, grid, block, 0, stream, start, n, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int A>
static hipError_t launch_a(const uint8_t *msgs, const uint64_t *offs, const uint64_t *lens, uint64_t n,
                           bool fixed, uint64_t fixed_len, uint8_t *out, uint32_t stride,
                           const uint8_t *filter, hipStream_t stream)
{
    const uint64_t blocks = (n + kPlainBlock - 1) / kPlainBlock;
    if (blocks > 0x7fffffffull) return hipErrorInvalidConfiguration;
    const dim3 grid{uint32_t(blocks), 1, 1}, block{kPlainBlock, 1, 1};
    if (fixed)
        hipLaunchKernelGGL((k_plain<A, true>), grid, block, 0, stream, msgs, offs, lens, n, fixed_len, out,
                           stride, filter);
    else
        hipLaunchKernelGGL((k_plain<A, false>), grid, block, 0, stream, msgs, offs, lens, n, fixed_len, out,
                           stride, filter);
    return hipGetLastError();
}

template <int A>
static hipError_t launch_lds_a(const uint8_t *msgs, uint64_t n, uint64_t len, uint8_t *out, hipStream_t stream)
{
    const uint64_t blocks = (n + kPlainBlock - 1) / kPlainBlock;
    if (blocks > 0x7fffffffull) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_plain_lds<A>, dim3(uint32_t(blocks)), dim3(kPlainBlock), 0, stream, msgs, n, len, out);
    return hipGetLastError();
}

bool plain_lds_applies(const uint8_t *msgs, uint64_t fixed_len, uint32_t stride, int algo)
{
    // all three algorithms by default; HB_PLAIN_LDS=0 keeps them per lane
    const char *v = std::getenv("HB_PLAIN_LDS");
    if (v && std::atoi(v) == 0) return false;
    // dword-aligned messages; 64 messages' offsets fit the loads' 32-bit offsets; packed digests
    return (reinterpret_cast<uintptr_t>(msgs) & 3u) == 0 && fixed_len % 4u == 0 && fixed_len > 0 &&
           fixed_len < (1ull << 25) && stride == uint32_t(digest_size(algo));
}

hipError_t launch_plain(int algo, const uint8_t *msgs, const uint64_t *offs, const uint64_t *lens,
                        uint64_t n, bool fixed, uint64_t fixed_len, uint8_t *out, uint32_t stride,
                        const uint8_t *filter, hipStream_t stream)
{
    if (fixed && !filter && plain_lds_applies(msgs, fixed_len, stride, algo)) {
        switch (algo) {
        case MD5: return launch_lds_a<MD5>(msgs, n, fixed_len, out, stream);
        case SHA1: return launch_lds_a<SHA1>(msgs, n, fixed_len, out, stream);
        case SM3: return launch_lds_a<SM3>(msgs, n, fixed_len, out, stream);
        default: return hipErrorInvalidValue;
        }
    }
    switch (algo) {
    case MD5: return launch_a<MD5>(msgs, offs, lens, n, fixed, fixed_len, out, stride, filter, stream);
    case SHA1: return launch_a<SHA1>(msgs, offs, lens, n, fixed, fixed_len, out, stride, filter, stream);
    case SM3: return launch_a<SM3>(msgs, offs, lens, n, fixed, fixed_len, out, stride, filter, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hb
