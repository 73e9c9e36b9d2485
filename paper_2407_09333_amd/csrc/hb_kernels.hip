// hb_kernels.hip -- plain batch-hashing kernels: one lane per message, in index order.
#include <algorithm>

#include "hb_device.hpp"
#include "hb_internal.hpp"

namespace hb {

constexpr int kPlainBlock = 256;

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
    const uint64_t i = uint64_t(blockIdx.x) * kPlainBlock + threadIdx.x;
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

hipError_t launch_plain(int algo, const uint8_t *msgs, const uint64_t *offs, const uint64_t *lens,
                        uint64_t n, bool fixed, uint64_t fixed_len, uint8_t *out, uint32_t stride,
                        const uint8_t *filter, hipStream_t stream)
{
    switch (algo) {
    case MD5: return launch_a<MD5>(msgs, offs, lens, n, fixed, fixed_len, out, stride, filter, stream);
    case SHA1: return launch_a<SHA1>(msgs, offs, lens, n, fixed, fixed_len, out, stride, filter, stream);
    case SM3: return launch_a<SM3>(msgs, offs, lens, n, fixed, fixed_len, out, stride, filter, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hb
