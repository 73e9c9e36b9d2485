// hb_kernels.hip -- plain batch-hashing kernels: one lane per message, in index order.
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
