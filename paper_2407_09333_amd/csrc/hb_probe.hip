// hb_probe.hip -- measures the integer-VALU issue rates the roofline is priced with.
//
// Every CU is filled with `wps` workgroups of four waves (wps waves per SIMD).  An
// instruction kind runs as long unrolled chains over eight independent accumulators per
// lane, so no instruction waits for the one before it; a compression kind runs the
// library's own compress<A> on register data with no memory traffic.  Each workgroup's
// first lane records s_memtime (engine cycles) and s_memrealtime (100 MHz) around its loop;
// the host turns the span of all workgroups into SIMD cycles per wave instruction (or per
// wave and 64-byte block).  Writes go only to the timestamp buffer (four words per
// workgroup) and one sink word per thread.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/hb.h"
#include "hb_device.hpp"
#include "hb_internal.hpp"

namespace hb {

namespace {

constexpr int kProbeThreads = 256;  // four waves: one per SIMD
constexpr int kProbeReps = 512;     // chunks of 64 instructions per wave
constexpr int kProbeBlocks = 256;   // compressions per lane

// One instruction per accumulator: %0..%7 accumulators, %8 and %9 the other operands.
#define HB_PR_ADD3(i) "v_add3_u32 %" #i ", %" #i ", %8, %9\n\t"
#define HB_PR_ALIGNBIT(i) "v_alignbit_b32 %" #i ", %" #i ", %" #i ", 7\n\t"
#define HB_PR_BITOP3(i) "v_bitop3_b32 %" #i ", %" #i ", %8, %9 bitop3:0x96\n\t"
#define HB_PR_ADD(i) "v_add_u32 %" #i ", %" #i ", %8\n\t"
#define HB_PR_XOR(i) "v_xor_b32 %" #i ", %" #i ", %8\n\t"
#define HB_PR_XAD(i) "v_xad_u32 %" #i ", %" #i ", %8, %9\n\t"
#define HB_PR_PERM(i) "v_perm_b32 %" #i ", %" #i ", %8, %9\n\t"
#define HB_PR_8(F) F(0) F(1) F(2) F(3) F(4) F(5) F(6) F(7)
// mixes: bitop3 and alignbit alternating; two bitop3 to one alignbit (eight accumulators,
// the pattern continuing across the 8-instruction groups of the .rept)
#define HB_PR_ALT HB_PR_BITOP3(0) HB_PR_ALIGNBIT(1) HB_PR_BITOP3(2) HB_PR_ALIGNBIT(3) \
                  HB_PR_BITOP3(4) HB_PR_ALIGNBIT(5) HB_PR_BITOP3(6) HB_PR_ALIGNBIT(7)
#define HB_PR_TWO_ONE HB_PR_BITOP3(0) HB_PR_BITOP3(1) HB_PR_ALIGNBIT(2) HB_PR_BITOP3(3) \
                      HB_PR_BITOP3(4) HB_PR_ALIGNBIT(5) HB_PR_BITOP3(6) HB_PR_BITOP3(7) \
                      HB_PR_ALIGNBIT(0) HB_PR_BITOP3(1) HB_PR_BITOP3(2) HB_PR_ALIGNBIT(3)
#define HB_PR_ASM(BODY, REPT)                                                                      \
    asm volatile(".rept " #REPT "\n\t" BODY ".endr"                                              \
                 : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]),      \
                   "+v"(a[6]), "+v"(a[7])                                                         \
                 : "v"(x), "v"(y))

// 64 instructions of kind K (the 2:1 mix: 12 per group, 60 in all, counted by the host)
template <int K> __device__ __forceinline__ void probe_chunk(uint32_t *a, uint32_t x, uint32_t y)
{
    if constexpr (K == HB_PROBE_ADD3) HB_PR_ASM(HB_PR_8(HB_PR_ADD3), 8);
    else if constexpr (K == HB_PROBE_ALIGNBIT) HB_PR_ASM(HB_PR_8(HB_PR_ALIGNBIT), 8);
    else if constexpr (K == HB_PROBE_BITOP3) HB_PR_ASM(HB_PR_8(HB_PR_BITOP3), 8);
    else if constexpr (K == HB_PROBE_ADD) HB_PR_ASM(HB_PR_8(HB_PR_ADD), 8);
    else if constexpr (K == HB_PROBE_XOR) HB_PR_ASM(HB_PR_8(HB_PR_XOR), 8);
    else if constexpr (K == HB_PROBE_XAD) HB_PR_ASM(HB_PR_8(HB_PR_XAD), 8);
    else if constexpr (K == HB_PROBE_PERM) HB_PR_ASM(HB_PR_8(HB_PR_PERM), 8);
    else if constexpr (K == HB_PROBE_MIX_ALT) HB_PR_ASM(HB_PR_ALT, 8);
    else HB_PR_ASM(HB_PR_TWO_ONE, 5);
}

template <int K> constexpr int chunk_instructions() { return K == HB_PROBE_MIX_2_1 ? 60 : 64; }

__device__ __forceinline__ void stamp(uint64_t *ts, uint64_t t0, uint64_t r0)
{
    const uint64_t t1 = __builtin_amdgcn_s_memtime(), r1 = __builtin_amdgcn_s_memrealtime();
    if (threadIdx.x == 0) {
        ts[4 * blockIdx.x] = t0;
        ts[4 * blockIdx.x + 1] = t1;
        ts[4 * blockIdx.x + 2] = r0;
        ts[4 * blockIdx.x + 3] = r1;
    }
}

template <int K> __global__ __launch_bounds__(kProbeThreads) void k_probe_instr(uint64_t *ts, uint32_t *sink, uint32_t seed)
{
    uint32_t a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = seed + threadIdx.x * uint32_t(k + 1);
    const uint32_t x = seed ^ 0x9e3779b9u, y = 0x03020100u + threadIdx.x;
    const uint64_t t0 = __builtin_amdgcn_s_memtime(), r0 = __builtin_amdgcn_s_memrealtime();
    for (int r = 0; r < kProbeReps; ++r) probe_chunk<K>(a, x, y);
    stamp(ts, t0, r0);
    uint32_t z = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) z ^= a[k];
    sink[blockIdx.x * kProbeThreads + threadIdx.x] = z;
}

// the library's compression on register data; one xor per block feeds the state back into
// the words so nothing is loop-invariant
template <int A> __global__ __launch_bounds__(kProbeThreads) void k_probe_compress(uint64_t *ts, uint32_t *sink, uint32_t seed)
{
    uint32_t w[16], s[8];
#pragma unroll
    for (int i = 0; i < 16; ++i) w[i] = seed * uint32_t(i + 1) + threadIdx.x * 0x85ebca6bu + blockIdx.x;
    init_state<A>(s);
    const uint64_t t0 = __builtin_amdgcn_s_memtime(), r0 = __builtin_amdgcn_s_memrealtime();
    for (int b = 0; b < kProbeBlocks; ++b) {
        compress<A>(s, w);
        w[b & 15] ^= s[0];
    }
    stamp(ts, t0, r0);
    uint32_t z = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) z ^= s[i];
    sink[blockIdx.x * kProbeThreads + threadIdx.x] = z;
}

template <int K> void launch_probe(int blocks, uint64_t *ts, uint32_t *sink, uint32_t seed)
{
    if constexpr (K <= HB_PROBE_MIX_2_1)
        hipLaunchKernelGGL(k_probe_instr<K>, dim3(uint32_t(blocks)), dim3(kProbeThreads), 0, 0, ts, sink, seed);
    else
        hipLaunchKernelGGL(k_probe_compress<K - HB_PROBE_MD5>, dim3(uint32_t(blocks)), dim3(kProbeThreads), 0, 0, ts,
                           sink, seed);
}

// units (wave instructions or wave-blocks) one wave runs
template <int K> constexpr double units_per_wave()
{
    if constexpr (K <= HB_PROBE_MIX_2_1) return double(kProbeReps) * chunk_instructions<K>();
    else return double(kProbeBlocks);
}

template <int K> int run_probe(int blocks, int cus, uint64_t *ts, uint32_t *sink, double *cycles, double *ghz)
{
    std::vector<uint64_t> h(size_t(blocks) * 4);
    double best = INFINITY, best_ghz = 0;
    for (int rep = 0; rep < 3; ++rep) {
        launch_probe<K>(blocks, ts, sink, 17u + uint32_t(rep));
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e == hipSuccess) e = hipMemcpy(h.data(), ts, h.size() * sizeof(uint64_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_error(e, "hb_probe_valu: probe launch");
        uint64_t rmin = ~0ull, rmax = 0;
        double cyc = 0, rt = 0;
        for (int b = 0; b < blocks; ++b) {
            rmin = std::min(rmin, h[4 * size_t(b) + 2]);
            rmax = std::max(rmax, h[4 * size_t(b) + 3]);
            cyc += double(h[4 * size_t(b) + 1] - h[4 * size_t(b)]);
            rt += double(h[4 * size_t(b) + 3] - h[4 * size_t(b) + 2]);
        }
        if (rt <= 0 || rmax <= rmin) return set_error(HB_EHIP, "hb_probe_valu: no elapsed time recorded");
        const double g = cyc / (rt * 10.0);                      // GHz: cycles per 10 ns tick
        const double simd_cycles = double(rmax - rmin) * 10.0 * g;  // span of all waves
        const double units_per_simd = double(blocks) * 4.0 * units_per_wave<K>() / (double(cus) * 4.0);
        const double c = simd_cycles / units_per_simd;
        if (c < best) { best = c; best_ghz = g; }
    }
    *cycles = best;
    if (ghz) *ghz = best_ghz;
    return HB_OK;
}

}  // namespace

}  // namespace hb

using namespace hb;

extern "C" int hb_probe_valu(int kind, int waves_per_simd, double *cycles_out, double *clock_ghz_out)
{
    if (kind < 0 || kind >= HB_PROBE_KINDS) return set_error(HB_EINVAL, "hb_probe_valu: unknown probe kind");
    if (waves_per_simd < 1 || waves_per_simd > 8) return set_error(HB_EINVAL, "hb_probe_valu: waves_per_simd must be 1..8");
    if (!cycles_out) return set_error(HB_EINVAL, "hb_probe_valu: null cycles_out");
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_error(e, "hb_probe_valu: device");
    const int blocks = cus * waves_per_simd;
    uint64_t *ts = nullptr;
    uint32_t *sink = nullptr;
    if ((e = hipMalloc(&ts, size_t(blocks) * 4 * sizeof(uint64_t))) != hipSuccess)
        return hip_error(e, "hb_probe_valu: hipMalloc");
    if ((e = hipMalloc(&sink, size_t(blocks) * kProbeThreads * sizeof(uint32_t))) != hipSuccess) {
        (void)hipFree(ts);
        return hip_error(e, "hb_probe_valu: hipMalloc");
    }
    int rc = HB_OK;
    switch (kind) {
    case HB_PROBE_ADD3: rc = run_probe<HB_PROBE_ADD3>(blocks, cus, ts, sink, cycles_out, clock_ghz_out); break;
    case HB_PROBE_ALIGNBIT: rc = run_probe<HB_PROBE_ALIGNBIT>(blocks, cus, ts, sink, cycles_out, clock_ghz_out); break;
    case HB_PROBE_BITOP3: rc = run_probe<HB_PROBE_BITOP3>(blocks, cus, ts, sink, cycles_out, clock_ghz_out); break;
    case HB_PROBE_ADD: rc = run_probe<HB_PROBE_ADD>(blocks, cus, ts, sink, cycles_out, clock_ghz_out); break;
    case HB_PROBE_XOR: rc = run_probe<HB_PROBE_XOR>(blocks, cus, ts, sink, cycles_out, clock_ghz_out); break;
    case HB_PROBE_XAD: rc = run_probe<HB_PROBE_XAD>(blocks, cus, ts, sink, cycles_out, clock_ghz_out); break;
    case HB_PROBE_PERM: rc = run_probe<HB_PROBE_PERM>(blocks, cus, ts, sink, cycles_out, clock_ghz_out); break;
    case HB_PROBE_MIX_ALT: rc = run_probe<HB_PROBE_MIX_ALT>(blocks, cus, ts, sink, cycles_out, clock_ghz_out); break;
    case HB_PROBE_MIX_2_1: rc = run_probe<HB_PROBE_MIX_2_1>(blocks, cus, ts, sink, cycles_out, clock_ghz_out); break;
    case HB_PROBE_MD5: rc = run_probe<HB_PROBE_MD5>(blocks, cus, ts, sink, cycles_out, clock_ghz_out); break;
    case HB_PROBE_SHA1: rc = run_probe<HB_PROBE_SHA1>(blocks, cus, ts, sink, cycles_out, clock_ghz_out); break;
    default: rc = run_probe<HB_PROBE_SM3>(blocks, cus, ts, sink, cycles_out, clock_ghz_out); break;
    }
    (void)hipFree(sink);
    (void)hipFree(ts);
    return rc;
}
