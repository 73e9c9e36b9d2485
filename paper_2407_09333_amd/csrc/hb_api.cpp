// hb_api.cpp -- C ABI entry points for the plain batch-hashing paths, error reporting and
// device facts.  Every argument error is reported before anything is enqueued.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/hb.h"
#include "hb_internal.hpp"

namespace hb {

static thread_local std::string g_last_error;

int set_error(int status, const std::string &msg)
{
    g_last_error = msg;
    return status;
}

int hip_error(hipError_t e, const char *what)
{
    return set_error(HB_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int digest_size(int algo)
{
    switch (algo) {
    case HB_MD5: return 16;
    case HB_SHA1: return 20;
    case HB_SM3: return 32;
    default: return 0;
    }
}

static int check_common(int algo, const void *messages, uint64_t n, const void *digests_out,
                        uint64_t stride, const char *fn)
{
    if (digest_size(algo) == 0)
        return set_error(HB_EINVAL, std::string(fn) + ": unknown algorithm id " + std::to_string(algo));
    if (n == 0) return HB_OK;
    if (!messages || !digests_out)
        return set_error(HB_EINVAL, std::string(fn) + ": null messages or digests_out pointer");
    if (reinterpret_cast<uintptr_t>(digests_out) & 3u)
        return set_error(HB_EINVAL, std::string(fn) + ": digests_out must be 4-byte aligned");
    if (stride % 4u || stride < uint64_t(digest_size(algo)) || stride > 0xffffffffull)
        return set_error(HB_EINVAL, std::string(fn) + ": stride must be a multiple of 4 and at least the digest size");
    return HB_OK;
}

}  // namespace hb

using namespace hb;

extern "C" {

size_t hb_digest_size(int algo) { return size_t(digest_size(algo)); }

const char *hb_last_error(void) { return g_last_error.c_str(); }

int hb_device_info(int *cu_count, int *wave_size, int *clock_khz, char *arch_name, size_t arch_len)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hb_device_info: hipGetDevice");
    hipDeviceProp_t p;
    e = hipGetDeviceProperties(&p, dev);
    if (e != hipSuccess) return hip_error(e, "hb_device_info: hipGetDeviceProperties");
    if (cu_count) *cu_count = p.multiProcessorCount;
    if (wave_size) *wave_size = p.warpSize;
    if (clock_khz) *clock_khz = p.clockRate;
    if (arch_name && arch_len) {
        std::snprintf(arch_name, arch_len, "%s", p.gcnArchName);
    }
    return HB_OK;
}

int hash_batch_strided(int algo, const uint8_t *messages, const uint64_t *offsets, const uint64_t *lengths,
                       uint64_t n, uint8_t *digests_out, uint64_t stride, void *stream)
{
    int rc = check_common(algo, messages, n, digests_out, stride, "hash_batch");
    if (rc != HB_OK || n == 0) return rc;
    if (!offsets || !lengths) return set_error(HB_EINVAL, "hash_batch: null offsets or lengths");
    hipError_t e = launch_plain(algo, messages, offsets, lengths, n, false, 0, digests_out, uint32_t(stride), nullptr,
                                static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HB_OK : hip_error(e, "hash_batch: launch");
}

int hash_batch(int algo, const uint8_t *messages, const uint64_t *offsets, const uint64_t *lengths, uint64_t n,
               uint8_t *digests_out, void *stream)
{
    return hash_batch_strided(algo, messages, offsets, lengths, n, digests_out, uint64_t(digest_size(algo)),
                              stream);
}

int hash_batch_fixed(int algo, const uint8_t *messages, uint64_t n, uint64_t msg_len, uint8_t *digests_out,
                     void *stream)
{
    const uint64_t ds = uint64_t(digest_size(algo));
    int rc = check_common(algo, messages, n, digests_out, ds, "hash_batch_fixed");
    if (rc != HB_OK || n == 0) return rc;
    if (msg_len >= (1ull << 61)) return set_error(HB_EINVAL, "hash_batch_fixed: msg_len must be below 2^61");
    hipError_t e = launch_plain(algo, messages, nullptr, nullptr, n, true, msg_len, digests_out, uint32_t(ds), nullptr,
                                static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HB_OK : hip_error(e, "hash_batch_fixed: launch");
}

int hash_batch_mixed(const uint8_t *algos, const uint8_t *messages, const uint64_t *offsets, const uint64_t *lengths,
                     uint64_t n, uint8_t *digests_out, void *stream)
{
    int rc = check_common(HB_MD5, messages, n, digests_out, 32, "hash_batch_mixed");
    if (rc != HB_OK || n == 0) return rc;
    if (!algos || !offsets || !lengths) return set_error(HB_EINVAL, "hash_batch_mixed: null algos, offsets or lengths");
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int a = HB_MD5; a <= HB_SM3; ++a) {
        hipError_t e = launch_plain(a, messages, offsets, lengths, n, false, 0, digests_out, 32u, algos, s);
        if (e != hipSuccess) return hip_error(e, "hash_batch_mixed: launch");
    }
    return HB_OK;
}

int hash_digits9(int algo, uint64_t start, uint64_t n, uint8_t *digests_out, void *stream)
{
    int rc = check_common(algo, digests_out ? digests_out : nullptr, n, digests_out, uint64_t(digest_size(algo)),
                          "hash_digits9");
    if (rc != HB_OK || n == 0) return rc;
    if (start >= 1000000000ull || n > 1000000000ull - start)
        return set_error(HB_EINVAL, "hash_digits9: start + n must not exceed 10^9 (nine decimal digits)");
    hipError_t e = launch_digits9(algo, start, n, digests_out, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HB_OK : hip_error(e, "hash_digits9: launch");
}

}  // extern "C"
