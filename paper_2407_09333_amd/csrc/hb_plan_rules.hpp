// hb_plan_rules.hpp -- sizing rules of the batched plan that the host can check without a
// GPU: block counts, sort keys, and the long-chain scratch region of a wave.  Free of HIP
// calls; compiled into the device kernels and into host-only checks alike.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__) || defined(__HIP__)
#define HB_HD __host__ __device__
#else
#define HB_HD
#endif

namespace hb {

constexpr uint32_t kBins = 16448;  // block-count keys per algorithm: key = min(nb, kBins - 1)

// Blocks of the padded L-byte message: the message, the 0x80 byte, zeros and the 8-byte
// length field fill floor((L + 8) / 64) + 1 blocks (RFC 1321 Sec. 3.1-3.2, FIPS 180-4
// Sec. 5.1.1, GB/T 32905 Sec. 5.2).
HB_HD inline uint64_t block_count(uint64_t len) { return (len + 8u) / 64u + 1u; }

// Sort key of an L-byte message: its block count, saturated at kBins - 1.  Every message
// of kBins - 1 blocks (about 1.05 MB) or more shares that key, so the bucketing sort leaves
// them in no particular order among themselves.
HB_HD inline uint32_t sort_key(uint64_t len)
{
    const uint64_t nb = block_count(len);
    return nb >= kBins ? kBins - 1 : uint32_t(nb);
}

// Scratch wave-blocks a long-chain wave needs: the largest block count among its `lanes`
// messages, len_at(l) giving lane l's length in sorted order.  Below the saturated key the
// sort is exact and descending, so lane 0 holds the largest; once lane 0's key is
// saturated the order is arbitrary and every lane is looked at.  The result is clamped to
// `limit`; a caller passing (scratch capacity + 1) reads `limit` as "cannot fit".
template <class LenAt>
HB_HD inline uint64_t wave_region_blocks(LenAt len_at, uint32_t lanes, uint64_t limit)
{
    const uint64_t len0 = len_at(0u);
    uint64_t r = block_count(len0);
    if (sort_key(len0) == kBins - 1)
        for (uint32_t l = 1; l < lanes; ++l) {
            const uint64_t b = block_count(len_at(l));
            r = b > r ? b : r;
        }
    return r < limit ? r : limit;
}

}  // namespace hb
