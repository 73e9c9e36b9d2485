// hb_internal.hpp -- host-side declarations shared by the libhb translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace hb {

// Thread-local last-error text (exposed by hb_last_error) and the status it goes with.
int set_error(int status, const std::string &msg);
int hip_error(hipError_t e, const char *what);

// Plain launches (one lane per message, index order).  `fixed` selects the contiguous
// fixed-length layout (message i at i * fixed_len; offsets/lengths unused).  filter !=
// nullptr hashes only the messages whose id equals algo (the MD5 launch also zeroes the
// slots of invalid ids).  Returns the hipError_t of the launch.
hipError_t launch_plain(int algo, const uint8_t *msgs, const uint64_t *offs, const uint64_t *lens,
                        uint64_t n, bool fixed, uint64_t fixed_len, uint8_t *out, uint32_t stride,
                        const uint8_t *filter, hipStream_t stream);

int digest_size(int algo);

// Hash messages [i0, i1) on host threads (the CPU share of a CPU + GPU split); message i's
// digest goes to out + (i - i0) * stride.  threads <= 0: all hardware threads.
void cpu_hash_range(const uint8_t *algos, int algo, const uint8_t *msgs, const uint64_t *offs, const uint64_t *lens,
                    uint64_t i0, uint64_t i1, uint8_t *out, uint32_t stride, int threads);

// Copy `bytes` between device-accessible buffers with a kernel on `stream` (no copy
// engine): device memory, or pinned host memory through its device mapping.
hipError_t launch_copy(void *dst, const void *src, uint64_t bytes, hipStream_t stream);

struct ServeRings;

// The resident serving kernel (hb_serve.hip): `workgroups` workgroups of 256 lanes, the
// first wave dispatching, the rest hashing published items until told to stop or idle.
hipError_t launch_serve(const ServeRings &rings, uint32_t gen, int workgroups, hipStream_t stream);

// The paper's 9-digit decimal workload, generated on the device (see hash_digits9).
hipError_t launch_digits9(int algo, uint64_t start, uint64_t n, uint8_t *out, hipStream_t stream);

}  // namespace hb
