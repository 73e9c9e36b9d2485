// hb_stream.hip -- incremental hashing of many messages: per-message chaining state that
// lives in device memory between launches (init / update / final).
//
// The paper's crypto dialect has a single-message op beside the multi-message one
// (Sec. IV-B); here both are the same batch kernels with n = 1 allowed.  Splitting a
// message into pieces lets a very long message span several launches (its chain can be
// suspended and resumed, and the state can be copied out and back in); the digest is the
// one of the whole message because the padding's length field counts every byte absorbed.
#include "../../include/hb.h"
#include "hb_device.hpp"
#include "hb_internal.hpp"

namespace hb {

constexpr int kStreamBlock = 256;
constexpr uint64_t kInvalidState = 1;  // hb_state.flags: a piece was not whole blocks

static_assert(sizeof(hb_state) == 48, "hb_state layout");

template <int A>
__global__ __launch_bounds__(kStreamBlock) void k_init(hb_state *__restrict__ st, uint64_t n)
{
    const uint64_t i = uint64_t(blockIdx.x) * kStreamBlock + threadIdx.x;
    if (i >= n) return;
    uint32_t s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    init_state<A>(s);
    for (int q = 0; q < 8; ++q) st[i].h[q] = s[q];
    st[i].bytes = 0;
    st[i].flags = 0;
}

template <int A>
__global__ __launch_bounds__(kStreamBlock) void k_update(hb_state *__restrict__ st, const uint8_t *__restrict__ msgs,
                                                         const uint64_t *__restrict__ offs,
                                                         const uint64_t *__restrict__ lens, uint64_t n)
{
    const uint64_t i = uint64_t(blockIdx.x) * kStreamBlock + threadIdx.x;
    if (i >= n) return;
    const uint64_t len = lens[i];
    if (st[i].flags) return;
    if (len % 64u) {  // only whole blocks can be absorbed before the final piece
        st[i].flags = kInvalidState;
        return;
    }
    uint32_t s[8];
    for (int q = 0; q < 8; ++q) s[q] = st[i].h[q];
    const Msg m = make_msg<A>(msgs + offs[i], len);
    absorb<A, false>(m, s);
    for (int q = 0; q < Traits<A>::kWords; ++q) st[i].h[q] = s[q];
    st[i].bytes += len;
}

template <int A>
__global__ __launch_bounds__(kStreamBlock) void k_final(const hb_state *__restrict__ st, const uint8_t *__restrict__ msgs,
                                                        const uint64_t *__restrict__ offs,
                                                        const uint64_t *__restrict__ lens, uint64_t n,
                                                        uint8_t *__restrict__ out)
{
    const uint64_t i = uint64_t(blockIdx.x) * kStreamBlock + threadIdx.x;
    if (i >= n) return;
    uint8_t *o = out + i * Traits<A>::kDigest;
    if (st[i].flags) {
        HB_GLOBAL uint32_t *ow = reinterpret_cast<HB_GLOBAL uint32_t *>(reinterpret_cast<uintptr_t>(o));
        for (int q = 0; q < Traits<A>::kWords; ++q) ow[q] = 0u;
        return;
    }
    uint32_t s[8];
    for (int q = 0; q < 8; ++q) s[q] = st[i].h[q];
    const uint64_t len = lens[i];
    Msg m = make_msg<A>(msgs + offs[i], len);
    m.bits = (st[i].bytes + len) << 3;
    absorb<A, true>(m, s);
    store_digest<A>(o, s, Traits<A>::kDigest);
}

template <class K, class... Args>
static hipError_t launch_n(K kernel, uint64_t n, hipStream_t stream, Args... args)
{
    const uint64_t blocks = (n + kStreamBlock - 1) / kStreamBlock;
    if (blocks > 0x7fffffffull) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(kernel, dim3(uint32_t(blocks)), dim3(kStreamBlock), 0, stream, args...);
    return hipGetLastError();
}

static int check_states(int algo, const void *states, uint64_t n, const char *fn)
{
    if (digest_size(algo) == 0) return set_error(HB_EINVAL, std::string(fn) + ": unknown algorithm id");
    if (n && !states) return set_error(HB_EINVAL, std::string(fn) + ": null states");
    if (reinterpret_cast<uintptr_t>(states) & 7u) return set_error(HB_EINVAL, std::string(fn) + ": states must be 8-byte aligned");
    return HB_OK;
}

}  // namespace hb

using namespace hb;

extern "C" {

int hash_init_batch(int algo, hb_state *states, uint64_t n, void *stream)
{
    int rc = check_states(algo, states, n, "hash_init_batch");
    if (rc != HB_OK || n == 0) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = algo == HB_MD5 ? launch_n(k_init<MD5>, n, s, states, n)
                 : algo == HB_SHA1 ? launch_n(k_init<SHA1>, n, s, states, n)
                                   : launch_n(k_init<SM3>, n, s, states, n);
    return e == hipSuccess ? HB_OK : hip_error(e, "hash_init_batch: launch");
}

int hash_update_batch(int algo, hb_state *states, const uint8_t *messages, const uint64_t *offsets,
                      const uint64_t *lengths, uint64_t n, void *stream)
{
    int rc = check_states(algo, states, n, "hash_update_batch");
    if (rc != HB_OK || n == 0) return rc;
    if (!messages || !offsets || !lengths) return set_error(HB_EINVAL, "hash_update_batch: null device pointer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = algo == HB_MD5 ? launch_n(k_update<MD5>, n, s, states, messages, offsets, lengths, n)
                 : algo == HB_SHA1 ? launch_n(k_update<SHA1>, n, s, states, messages, offsets, lengths, n)
                                   : launch_n(k_update<SM3>, n, s, states, messages, offsets, lengths, n);
    return e == hipSuccess ? HB_OK : hip_error(e, "hash_update_batch: launch");
}

int hash_final_batch(int algo, const hb_state *states, const uint8_t *messages, const uint64_t *offsets,
                     const uint64_t *lengths, uint64_t n, uint8_t *digests_out, void *stream)
{
    int rc = check_states(algo, states, n, "hash_final_batch");
    if (rc != HB_OK || n == 0) return rc;
    if (!messages || !offsets || !lengths || !digests_out)
        return set_error(HB_EINVAL, "hash_final_batch: null device pointer");
    if (reinterpret_cast<uintptr_t>(digests_out) & 3u)
        return set_error(HB_EINVAL, "hash_final_batch: digests_out must be 4-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = algo == HB_MD5 ? launch_n(k_final<MD5>, n, s, states, messages, offsets, lengths, n, digests_out)
                 : algo == HB_SHA1 ? launch_n(k_final<SHA1>, n, s, states, messages, offsets, lengths, n, digests_out)
                                   : launch_n(k_final<SM3>, n, s, states, messages, offsets, lengths, n, digests_out);
    return e == hipSuccess ? HB_OK : hip_error(e, "hash_final_batch: launch");
}

}  // extern "C"
