// hb_host.cpp -- hashing messages that live in host memory.
//
// The batch is cut into chunks of about chunk_bytes of payload.  For each chunk the host
// packs its messages (and rebased offsets, lengths, ids) into one of two pinned staging
// buffers; the copy stream moves it to one of two device buffers; the compute stream waits
// on the copy's event and runs the bucketed plan over the chunk; a kernel on the compute
// stream writes the digests into pinned memory.  While chunk k is hashed, chunk k+1 is
// packed and copied.  A small batch skips the copies: it is packed once and hashed where
// it lies in pinned memory (zero-copy), the digests written straight to pinned memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "../../include/hb.h"
#include "hb_internal.hpp"

namespace hb {

namespace {

struct Slot {
    uint8_t *h_msgs = nullptr;       // pinned staging: payload | offsets | lengths | ids
    uint64_t *h_offs = nullptr, *h_lens = nullptr;
    uint8_t *h_ids = nullptr;
    uint8_t *h_dig = nullptr;        // pinned digests
    uint8_t *m_dig = nullptr;        // the same, through its device mapping
    uint8_t *d_msgs = nullptr;
    uint64_t *d_offs = nullptr, *d_lens = nullptr;
    uint8_t *d_ids = nullptr, *d_dig = nullptr;
    uint64_t cap_bytes = 0, cap_n = 0;
    hipEvent_t copied = nullptr, drained = nullptr;
    // chunk bookkeeping for the drain step
    uint64_t first = 0, count = 0;
    bool busy = false;
};

struct HostPipe {
    int device = -1;
    hipStream_t copy = nullptr, compute = nullptr;  // H2D; hashing and the digest write-back
    Slot slot[2];
    // Two plans, both kept between calls and neither with a stream of its own: one
    // without the long-chain path and one with it, in one launch with the bulk (it also
    // holds the long-chain scratch, HB_LONG_SCRATCH_MB).  The host sees every length, so
    // it knows which one a batch needs.
    hb_plan *plan = nullptr, *plan_long = nullptr;
    uint64_t plan_n = 0, plan_long_n = 0;

    ~HostPipe()
    {
        if (compute) hipStreamSynchronize(compute);
        if (copy) hipStreamSynchronize(copy);
        for (Slot &s : slot) release(s);
        if (plan) hb_plan_destroy(plan);
        if (plan_long) hb_plan_destroy(plan_long);
        if (copy) hipStreamDestroy(copy);
        if (compute) hipStreamDestroy(compute);
    }

    void release_streams()
    {
        if (compute) { hipStreamSynchronize(compute); hipStreamDestroy(compute); compute = nullptr; }
        if (copy) { hipStreamSynchronize(copy); hipStreamDestroy(copy); copy = nullptr; }
    }

    static void release(Slot &s)
    {
        if (s.h_msgs) hipHostFree(s.h_msgs);
        if (s.h_dig) hipHostFree(s.h_dig);
        if (s.d_msgs) hipFree(s.d_msgs);
        if (s.copied) hipEventDestroy(s.copied);
        if (s.drained) hipEventDestroy(s.drained);
        s = Slot{};
    }
};

thread_local std::unique_ptr<HostPipe> t_pipe;

uint64_t up256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// Batches of at most this much payload (and at most kZeroCopyMaxN messages) are hashed
// straight from pinned host memory: one plain launch reads the packed messages and writes
// the digests over the host link, with no copy-engine transfer and no bucketing.
// HB_HOST_ZERO_COPY_MAX (bytes; 0 turns the path off) overrides the payload limit.
constexpr uint64_t kZeroCopyMax = 16ull << 20;
constexpr uint64_t kZeroCopyMaxN = 1ull << 20;

uint64_t zero_copy_max()
{
    if (const char *v = std::getenv("HB_HOST_ZERO_COPY_MAX")) return std::strtoull(v, nullptr, 10);
    return kZeroCopyMax;
}

// memcpy split over up to 8 threads for large copies into pinned staging.
void copy_parallel(uint8_t *dst, const uint8_t *src, uint64_t n)
{
    constexpr uint64_t kPer = 8ull << 20;
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const uint64_t parts = std::min<uint64_t>({(n + kPer - 1) / kPer, 8, hw});
    if (parts <= 1) {
        std::memcpy(dst, src, n);
        return;
    }
    std::vector<std::thread> th;
    const uint64_t step = (n + parts - 1) / parts;
    for (uint64_t k = 1; k < parts; ++k) {
        const uint64_t a = k * step, b = std::min(n, a + step);
        if (a < b) th.emplace_back([=] { std::memcpy(dst + a, src + a, b - a); });
    }
    std::memcpy(dst, src, std::min(n, step));
    for (auto &t : th) t.join();
}

// Make sure slot s holds at least `bytes` of payload and `n` messages.
int ensure_slot(Slot &s, uint64_t bytes, uint64_t n)
{
    if (s.cap_bytes >= bytes && s.cap_n >= n && s.h_msgs) return HB_OK;
    HostPipe::release(s);
    bytes = std::max<uint64_t>(up256(bytes), 1 << 20);
    n = std::max<uint64_t>(n, 4096);
    const uint64_t meta = up256(n * 8) * 2 + up256(n);
    const uint64_t total = bytes + meta;
    hipError_t e;
    if ((e = hipHostMalloc(reinterpret_cast<void **>(&s.h_msgs), total, hipHostMallocDefault)) != hipSuccess)
        return set_error(HB_ENOMEM, "hash_batch_host: pinned staging allocation failed");
    if ((e = hipHostMalloc(reinterpret_cast<void **>(&s.h_dig), n * 32, hipHostMallocMapped | hipHostMallocCoherent)) !=
        hipSuccess)
        return set_error(HB_ENOMEM, "hash_batch_host: pinned digest allocation failed");
    if ((e = hipHostGetDevicePointer(reinterpret_cast<void **>(&s.m_dig), s.h_dig, 0)) != hipSuccess)
        return hip_error(e, "hash_batch_host: device mapping of pinned digests");
    void *d = nullptr;
    if ((e = hipMalloc(&d, total + n * 32)) != hipSuccess)
        return set_error(HB_ENOMEM, "hash_batch_host: device staging allocation failed");
    s.d_msgs = static_cast<uint8_t *>(d);
    s.h_offs = reinterpret_cast<uint64_t *>(s.h_msgs + bytes);
    s.h_lens = reinterpret_cast<uint64_t *>(s.h_msgs + bytes + up256(n * 8));
    s.h_ids = s.h_msgs + bytes + 2 * up256(n * 8);
    s.d_offs = reinterpret_cast<uint64_t *>(s.d_msgs + bytes);
    s.d_lens = reinterpret_cast<uint64_t *>(s.d_msgs + bytes + up256(n * 8));
    s.d_ids = s.d_msgs + bytes + 2 * up256(n * 8);
    s.d_dig = s.d_msgs + total;
    s.cap_bytes = bytes;
    s.cap_n = n;
    if ((e = hipEventCreateWithFlags(&s.copied, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&s.drained, hipEventDisableTiming)) != hipSuccess)
        return hip_error(e, "hash_batch_host: events");
    return HB_OK;
}

// Pack messages [i0, i1) into slot s (payload back to back, rebased offsets, lengths, ids);
// returns the payload bytes.
uint64_t pack_chunk(Slot &s, const uint8_t *algos_host, const uint8_t *messages_host, const uint64_t *offsets_host,
                    const uint64_t *lengths_host, uint64_t i0, uint64_t i1)
{
    uint64_t pos = 0;
    // a run of back-to-back messages is copied as one range
    bool packed = true;
    for (uint64_t i = i0; i < i1; ++i) {
        const uint64_t L = lengths_host[i];
        if (i > i0 && offsets_host[i] != offsets_host[i - 1] + lengths_host[i - 1]) packed = false;
        s.h_offs[i - i0] = pos;
        s.h_lens[i - i0] = L;
        if (algos_host) s.h_ids[i - i0] = algos_host[i];
        pos += L;
    }
    if (packed) {
        if (pos) copy_parallel(s.h_msgs, messages_host + offsets_host[i0], pos);
    } else {
        for (uint64_t i = i0; i < i1; ++i)
            if (lengths_host[i]) std::memcpy(s.h_msgs + s.h_offs[i - i0], messages_host + offsets_host[i], lengths_host[i]);
    }
    return pos;
}

// Small batch: pack into pinned staging, hash it where it is (the kernels read and write
// pinned host memory through its device mapping), copy the digests out.
int hash_small_zero_copy(HostPipe &P, const uint8_t *algos_host, int algo, const uint8_t *messages_host,
                         const uint64_t *offsets_host, const uint64_t *lengths_host, uint64_t n,
                         uint8_t *digests_out_host, uint64_t total_bytes)
{
    Slot &s = P.slot[0];
    int rc = ensure_slot(s, total_bytes, n);
    if (rc != HB_OK) return rc;
    hipError_t e = hipSuccess;
    if (!P.compute && (e = hipStreamCreateWithFlags(&P.compute, hipStreamNonBlocking)) != hipSuccess)
        return hip_error(e, "hash_batch_host: stream");
    pack_chunk(s, algos_host, messages_host, offsets_host, lengths_host, 0, n);
    void *dm = nullptr;
    if ((e = hipHostGetDevicePointer(&dm, s.h_msgs, 0)) != hipSuccess)
        return hip_error(e, "hash_batch_host: device mapping of pinned staging");
    // the staging block is one allocation: payload | offsets | lengths | ids
    uint8_t *d_msgs = static_cast<uint8_t *>(dm);
    const uint64_t *d_offs = reinterpret_cast<const uint64_t *>(d_msgs + (reinterpret_cast<uint8_t *>(s.h_offs) - s.h_msgs));
    const uint64_t *d_lens = reinterpret_cast<const uint64_t *>(d_msgs + (reinterpret_cast<uint8_t *>(s.h_lens) - s.h_msgs));
    const uint8_t *d_ids = d_msgs + (s.h_ids - s.h_msgs);
    uint8_t *d_dig = s.m_dig;
    const uint32_t stride = algos_host ? 32u : uint32_t(digest_size(algo));
    if (algos_host) {
        for (int a = 0; a < 3 && e == hipSuccess; ++a)
            e = launch_plain(a, d_msgs, d_offs, d_lens, n, false, 0, d_dig, stride, d_ids, P.compute);
    } else {
        e = launch_plain(algo, d_msgs, d_offs, d_lens, n, false, 0, d_dig, stride, nullptr, P.compute);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(P.compute);
    if (e != hipSuccess) return hip_error(e, "hash_batch_host: zero-copy hash");
    std::memcpy(digests_out_host, s.h_dig, n * stride);
    P.release_streams();
    return HB_OK;
}

}  // namespace

}  // namespace hb

using namespace hb;

extern "C" int hash_batch_host(const uint8_t *algos_host, int algo, const uint8_t *messages_host,
                               const uint64_t *offsets_host, const uint64_t *lengths_host, uint64_t n,
                               uint8_t *digests_out_host, uint64_t chunk_bytes)
{
    if (!algos_host && digest_size(algo) == 0) return set_error(HB_EINVAL, "hash_batch_host: unknown algorithm id");
    if (n == 0) return HB_OK;
    if (!offsets_host || !lengths_host || !digests_out_host)
        return set_error(HB_EINVAL, "hash_batch_host: null host pointer");
    if (chunk_bytes == 0) chunk_bytes = 64ull << 20;
    const uint64_t stride = algos_host ? 32 : uint64_t(digest_size(algo));
    uint64_t any_bytes = 0, total_bytes = 0;
    for (uint64_t i = 0; i < n; ++i) {
        if (lengths_host[i] >= (1ull << 61)) return set_error(HB_EINVAL, "hash_batch_host: length beyond 2^61");
        any_bytes |= lengths_host[i];
        total_bytes += lengths_host[i];
    }
    if (any_bytes && !messages_host) return set_error(HB_EINVAL, "hash_batch_host: null messages");

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hash_batch_host: hipGetDevice");
    if (!t_pipe || t_pipe->device != dev) {
        t_pipe.reset(new HostPipe());
        t_pipe->device = dev;
    }
    const bool zero_copy = total_bytes <= zero_copy_max() && n <= kZeroCopyMaxN;
    if (zero_copy) return hash_small_zero_copy(*t_pipe, algos_host, algo, messages_host, offsets_host, lengths_host, n,
                                               digests_out_host, total_bytes);
    if (!t_pipe->copy) {
        if ((e = hipStreamCreateWithFlags(&t_pipe->copy, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipStreamCreateWithFlags(&t_pipe->compute, hipStreamNonBlocking)) != hipSuccess) {
            t_pipe.reset();
            return hip_error(e, "hash_batch_host: streams");
        }
    }
    HostPipe &P = *t_pipe;
    const uint64_t max_chunk_n = 1ull << 22;

    // Chunk boundaries: greedy by payload bytes and message count.
    std::vector<uint64_t> cuts{0};
    uint64_t acc = 0, largest_chunk = 0, largest_n = 0;
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t L = lengths_host[i];
        if (i > cuts.back() && (acc + L > chunk_bytes || i - cuts.back() >= max_chunk_n)) {
            largest_chunk = std::max(largest_chunk, acc);
            largest_n = std::max(largest_n, i - cuts.back());
            cuts.push_back(i);
            acc = 0;
        }
        acc += L;
    }
    largest_chunk = std::max(largest_chunk, acc);
    largest_n = std::max(largest_n, n - cuts.back());
    cuts.push_back(n);

    // the long-chain path only pays off for messages of at least HB_LONG_MIN_BLOCKS blocks
    uint64_t long_blocks = 256;
    if (const char *v = std::getenv("HB_LONG_MIN_BLOCKS")) long_blocks = std::strtoull(v, nullptr, 10);
    uint64_t max_len = 0;
    for (uint64_t i = 0; i < n; ++i) max_len = std::max(max_len, lengths_host[i]);
    const bool want_long = (max_len + 8) / 64 + 1 >= long_blocks;
    hb_plan *&plan = want_long ? P.plan_long : P.plan;
    uint64_t &plan_n = want_long ? P.plan_long_n : P.plan_n;
    if (!plan || plan_n < largest_n) {
        if (plan) hb_plan_destroy(plan);
        plan = nullptr;
        int rc = hb_plan_create(&plan, std::max<uint64_t>(largest_n, 4096), want_long ? HB_PLAN_LONG_INLINE : HB_PLAN_NO_LONG);
        if (rc != HB_OK) return rc;
        plan_n = std::max<uint64_t>(largest_n, 4096);
    }
    for (Slot &s : P.slot) {
        int rc = ensure_slot(s, largest_chunk, largest_n);
        if (rc != HB_OK) return rc;
        s.busy = false;
    }

    auto drain = [&](Slot &s) -> int {
        if (!s.busy) return HB_OK;
        hipError_t de = hipEventSynchronize(s.drained);
        if (de != hipSuccess) return hip_error(de, "hash_batch_host: chunk");
        for (uint64_t k = 0; k < s.count; ++k)
            std::memcpy(digests_out_host + (s.first + k) * stride, s.h_dig + k * stride, stride);
        s.busy = false;
        return HB_OK;
    };

    int rc = HB_OK;
    const size_t nchunks = cuts.size() - 1;
    for (size_t c = 0; c < nchunks && rc == HB_OK; ++c) {
        Slot &s = P.slot[c & 1];
        rc = drain(s);  // the slot's previous chunk must be finished before its buffers are reused
        if (rc != HB_OK) break;
        const uint64_t i0 = cuts[c], i1 = cuts[c + 1], cnt = i1 - i0;
        const uint64_t pos = pack_chunk(s, algos_host, messages_host, offsets_host, lengths_host, i0, i1);
        const uint64_t bytes = pos;
        if (bytes) e = hipMemcpyAsync(s.d_msgs, s.h_msgs, bytes, hipMemcpyHostToDevice, P.copy);
        if (e == hipSuccess) e = hipMemcpyAsync(s.d_offs, s.h_offs, cnt * 8, hipMemcpyHostToDevice, P.copy);
        if (e == hipSuccess) e = hipMemcpyAsync(s.d_lens, s.h_lens, cnt * 8, hipMemcpyHostToDevice, P.copy);
        if (e == hipSuccess && algos_host) e = hipMemcpyAsync(s.d_ids, s.h_ids, cnt, hipMemcpyHostToDevice, P.copy);
        if (e == hipSuccess) e = hipEventRecord(s.copied, P.copy);
        if (e == hipSuccess) e = hipStreamWaitEvent(P.compute, s.copied, 0);
        if (e != hipSuccess) { rc = hip_error(e, "hash_batch_host: copy"); break; }
        rc = hb_plan_run(plan, algos_host ? s.d_ids : nullptr, algo, s.d_msgs, s.d_offs, s.d_lens, cnt, s.d_dig,
                         P.compute);
        if (rc != HB_OK) break;
        // digests go back by a kernel through the pinned buffer's device mapping: a
        // copy-engine transfer waiting on this chunk's hashing would hold up the next
        // chunk's payload copy
        e = launch_copy(s.m_dig, s.d_dig, cnt * stride, P.compute);
        if (e == hipSuccess) e = hipEventRecord(s.drained, P.compute);
        if (e != hipSuccess) { rc = hip_error(e, "hash_batch_host: digests"); break; }
        s.first = i0;
        s.count = cnt;
        s.busy = true;
    }
    for (Slot &s : P.slot) {
        int r2 = drain(s);
        if (rc == HB_OK) rc = r2;
    }
    // Release the streams between calls: each stream may hold one of the process's few
    // hardware queues, and idle streams still shift which queue later streams of the
    // caller (or of a serving loop) share.  Buffers and plans are kept.
    P.release_streams();
    return rc;
}

extern "C" int hash_batch_host_split(const uint8_t *algos_host, int algo, const uint8_t *messages_host,
                                     const uint64_t *offsets_host, const uint64_t *lengths_host, uint64_t n,
                                     uint8_t *digests_out_host, uint64_t chunk_bytes, double cpu_fraction,
                                     int cpu_threads)
{
    if (!algos_host && digest_size(algo) == 0)
        return set_error(HB_EINVAL, "hash_batch_host_split: unknown algorithm id");
    if (!(cpu_fraction >= 0.0 && cpu_fraction <= 1.0))
        return set_error(HB_EINVAL, "hash_batch_host_split: cpu_fraction must lie in [0, 1]");
    if (n == 0) return HB_OK;
    if (!offsets_host || !lengths_host || !digests_out_host)
        return set_error(HB_EINVAL, "hash_batch_host_split: null host pointer");
    uint64_t total = 0;
    for (uint64_t i = 0; i < n; ++i) {
        if (lengths_host[i] >= (1ull << 61)) return set_error(HB_EINVAL, "hash_batch_host_split: length beyond 2^61");
        total += lengths_host[i];
    }
    if (total && !messages_host) return set_error(HB_EINVAL, "hash_batch_host_split: null messages");
    // The host cores take the trailing messages holding about cpu_fraction of the payload
    // (work grows with bytes); the GPU pipeline takes the rest, both at once.
    uint64_t k = n;
    if (cpu_fraction >= 1.0) k = 0;
    else if (cpu_fraction > 0.0) {
        const double want = cpu_fraction * double(total);
        double tail = 0.0;
        while (k > 0 && tail + 0.5 * double(lengths_host[k - 1]) < want) tail += double(lengths_host[--k]);
    }
    const uint32_t stride = algos_host ? 32u : uint32_t(digest_size(algo));
    std::thread cpu;
    if (k < n)
        cpu = std::thread([=] {
            cpu_hash_range(algos_host, algo, messages_host, offsets_host, lengths_host, k, n,
                           digests_out_host + k * stride, stride, cpu_threads);
        });
    int rc = HB_OK;
    if (k > 0) rc = hash_batch_host(algos_host, algo, messages_host, offsets_host, lengths_host, k, digests_out_host,
                                    chunk_bytes);
    if (cpu.joinable()) cpu.join();
    return rc;
}
