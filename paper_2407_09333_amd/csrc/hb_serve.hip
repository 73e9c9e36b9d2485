// hb_serve.hip -- the resident serving kernel: requests join the device work already running.
//
// The serving loop publishes work items (up to 64 messages of one algorithm each) into a
// ring in pinned host memory as soon as a request's payload has landed in the device
// arena.  One launch of k_serve stays resident while items keep coming: its first wave is
// the dispatcher, which polls the host ring's tail over PCIe and copies new items into a
// device-memory ring; every other wave claims items from that ring with a compare-and-swap
// on the ring's head, hashes them (one lane per message, digests written straight to pinned
// host memory) and sets the item's done flag there.  So a request that arrives while long
// chains are being hashed starts on an idle wave at once instead of waiting for a step to
// end.  Every wave's wait is bounded: the dispatcher stops the launch after idle_ticks
// without a new item (or when the host sets its stop flag, or after max_ticks), every
// worker leaves when told to, or on its own after twice the idle time; the host relaunches
// when items are published and no launch is running.  Head and tail live in device memory
// across launches, so items a finished launch did not take are taken by the next.
#include "hb_device.hpp"
#include "hb_internal.hpp"
#include "hb_long.hpp"
#include "hb_plan_rules.hpp"
#include "hb_serve.hpp"

namespace hb {

constexpr uint64_t kMaxClaim = 16;  // items one wave claims at once at most
// s_waitcnt immediate: vmcnt(0), expcnt and lgkmcnt left at their maxima (gfx9 encoding:
// vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8)
constexpr int kWaitVmcnt0 = 0x0F70;

__device__ __forceinline__ uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }  // 100 MHz

__device__ __forceinline__ uint64_t bcast64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(v >> 32));
    return (uint64_t(hi) << 32) | lo;
}

// One item: lane l hashes message slot first + l.  The wave's 64 digests (32 bytes each,
// canonical bytes, zero past the digest size) are gathered in LDS and written to the digest
// ring's slots first .. first + count - 1 with whole 16-byte stores from consecutive lanes,
// so the writes cross PCIe as whole lines rather than as 4-byte pieces; the loop reorders
// them into the caller's order.  The item's algorithm is the same for every lane.
template <int A>
__device__ __forceinline__ void serve_lane(const ServeRings &R, uint32_t slot, uint32_t *mine)
{
    const uint64_t off = R.off[slot], len = R.len[slot];
    uint32_t s[8];
    if constexpr (A == MD5) hash_message<MD5>(R.arena + off, len, s);
    else hash_message_prefetch<A>(R.arena + off, len, s);
#pragma unroll
    for (int q = 0; q < 8; ++q)
        mine[q] = q < Traits<A>::kWords ? (Traits<A>::kBE ? bswap32(s[q]) : s[q]) : 0u;
}

// Long messages (an item of the longest block-count classes), the wave working together:
// the schedule words of up to 64 blocks -- `per` consecutive blocks of each of the item's
// `count` messages, one block per lane -- are computed into the wave's LDS window, then
// the lanes holding the messages run those blocks rounds only (SM3 921 instead of 1,350
// instructions per block, SHA-1 444 instead of 614, MD5 292 instead of 340), and the
// window moves on.  A chain is strictly sequential, so this shortens the item's critical
// path, which is what a request's latency is when it holds such a message.  LDS layout:
// word group g (4 words) of window entry e at sched[g][e], so the lanes reading one group
// of different entries hit consecutive 16-byte LDS slots.
template <int A>
__device__ __forceinline__ void serve_long_item(const ServeRings &R, const ServeItem &it, uint32_t lane,
                                                u32x4 (*sched)[64], uint32_t *mine)
{
    constexpr int N = SchedWords<A>::kN;
    const uint32_t count = it.count;
    const uint32_t per = 64u / count;  // window blocks per message (count <= 64)
    // each lane's own message (chain lanes), and the message whose block it schedules
    uint64_t off = 0, len = 0;
    if (lane < count) {
        off = R.off[it.first + lane];
        len = R.len[it.first + lane];
    }
    const uint32_t m = lane / per, j = lane % per;  // scheduled message and window block
    const uint32_t src = m < count ? m : 0u;
    const uint64_t m_off = __shfl(off, int(src)), m_len = __shfl(len, int(src));
    const uint64_t m_nb = block_count(m_len);
    uint64_t nb_max = lane < count ? block_count(len) : 0u;
    for (int d = 32; d >= 1; d >>= 1) {
        const uint64_t o = __shfl_xor(nb_max, d);
        nb_max = o > nb_max ? o : nb_max;
    }
    const Msg mm = make_msg<A>(R.arena + m_off, m_len);
    const uint64_t nb = block_count(len);
    uint32_t st[8];
    init_state<A>(st);
    for (uint64_t b0 = 0; b0 < nb_max; b0 += per) {
        const uint64_t blk = b0 + j;
        if (m < count && blk < m_nb) {
            uint32_t w[16], out[N];
            if (blk < m_len / 64u) load_full_block(mm, blk, w);
            else load_any_block<Traits<A>::kBE>(mm, blk, blk + 1 == m_nb, w);
            sched_block<A>(w, out);
#pragma unroll
            for (int g = 0; g < N / 4; ++g) sched[g][lane] = u32x4{out[4 * g], out[4 * g + 1], out[4 * g + 2], out[4 * g + 3]};
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the window's words before the chains read them
        if (lane < count) {
            for (uint32_t k = 0; k < per && b0 + k < nb; ++k) {
                uint32_t ww[N];
                const uint32_t e = lane * per + k;
#pragma unroll
                for (int g = 0; g < N / 4; ++g) {
                    const u32x4 v = sched[g][e];
                    ww[4 * g] = v.x; ww[4 * g + 1] = v.y; ww[4 * g + 2] = v.z; ww[4 * g + 3] = v.w;
                }
                rounds<A>(st, ww);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // chains done before the window is rewritten
    }
    if (lane < count) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
            mine[q] = q < Traits<A>::kWords ? (Traits<A>::kBE ? bswap32(st[q]) : st[q]) : 0u;
    }
}

__device__ __forceinline__ void serve_item(const ServeRings &R, const ServeItem &it, uint32_t lane, uint32_t *wave_lds,
                                           u32x4 (*sched)[64])
{
    uint32_t *mine = wave_lds + lane * 8u;
    if (it.blocks >= kServeCoopBlocks && it.count <= kServeCoopMaxMessages) {
        if (it.algo == MD5) serve_long_item<MD5>(R, it, lane, sched, mine);
        else if (it.algo == SHA1) serve_long_item<SHA1>(R, it, lane, sched, mine);
        else serve_long_item<SM3>(R, it, lane, sched, mine);
    } else if (lane < it.count) {
        if (it.algo == MD5) serve_lane<MD5>(R, it.first + lane, mine);
        else if (it.algo == SHA1) serve_lane<SHA1>(R, it.first + lane, mine);
        else serve_lane<SM3>(R, it.first + lane, mine);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the wave's LDS writes before its reads
    const uint32_t chunks = it.count * 2u;  // 16-byte chunks of the item's digests
    uint8_t *dst = R.digests + uint64_t(it.first) * 32u;
    for (uint32_t c = lane; c < chunks; c += 64u) {
        const uint32_t *src = wave_lds + c * 4u;
        u32x4 v;
        v.x = src[0]; v.y = src[1]; v.z = src[2]; v.w = src[3];
        // system-coherent 16-byte store (sc0 sc1), written through to pinned host memory
        // rather than held in the L2: the items' done flags then need these stores complete
        // (one vmcnt wait), not a write-back of the whole L2 per claim.  The compiler cannot
        // see this store, so the wait state the ISA asks before a VALU overwrites the data
        // registers of a store of more than 8 bytes is part of the asm.  (Four dword atomic
        // stores instead cut the serving rate more than tenfold.)
        HB_GLOBAL u32x4 *d = reinterpret_cast<HB_GLOBAL u32x4 *>(reinterpret_cast<uintptr_t>(dst + uint64_t(c) * 16u));
        asm volatile("global_store_dwordx4 %0, %1, off sc0 sc1\n\ts_nop 0" : : "v"(d), "v"(v) : "memory");
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // reads done before the next item's writes
}

__global__ __launch_bounds__(kServeThreads) void k_serve(ServeRings R, uint32_t gen)
{
    __shared__ uint32_t digest_lds[kServeThreads / 64][64 * 8];  // per wave: 64 digests of 32 bytes
    __shared__ u32x4 sched_lds[kServeThreads / 64][kSchedWords / 4][64];  // per wave: 64 blocks' words
    const uint32_t lane = __lane_id();
    const uint64_t mask = R.items_cap - 1u;
    const uint64_t t0 = now_ticks();
    if (blockIdx.x == 0 && threadIdx.x < 64) {
        // dispatcher: host ring -> device ring
        uint64_t dt = bcast64(lane == 0 ? __hip_atomic_load(R.d_tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0);
        uint64_t last = t0;
        for (;;) {
            const uint64_t now = now_ticks();
            uint64_t ht = 0, head = 0;
            uint32_t stop = 0;
            // relaxed polls: an acquire here would invalidate this XCD's L2 on every poll
            if (lane == 0) {
                stop = __hip_atomic_load(R.h_stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                ht = __hip_atomic_load(R.h_tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                head = __hip_atomic_load(R.d_head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            stop = __builtin_amdgcn_readfirstlane(stop);
            ht = bcast64(ht);
            head = bcast64(head);
            if (ht > dt) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // the host's item writes
                for (uint64_t k = dt + lane; k < ht; k += 64) R.d_items[k & mask] = R.h_items[k & mask];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                if (lane == 0) __hip_atomic_store(R.d_tail, ht, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                dt = ht;
                last = now;
            } else if (head < dt) {
                last = now;  // items still wait to be claimed
            }
            if (stop || now - last > R.idle_ticks || now - t0 > R.max_ticks) break;
            __builtin_amdgcn_s_sleep(8);
        }
        if (lane == 0) __hip_atomic_store(R.d_stop, gen, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    // workers: an idle wave polls the device ring's tail and stop word every ~2 us (one
    // lane, two relaxed loads: an acquire would invalidate the XCD's L2 on every poll), so a
    // thousand idle waves cost little; the one acquire is made after an item is claimed
    uint64_t last = t0;
    for (;;) {
        uint64_t h = 0, t = 0;
        uint32_t stop = 0;
        if (lane == 0) {
            stop = __hip_atomic_load(R.d_stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            t = __hip_atomic_load(R.d_tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        stop = __builtin_amdgcn_readfirstlane(stop);
        t = bcast64(t);
        if (stop == gen) break;
        if (lane == 0) h = __hip_atomic_load(R.d_head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        h = bcast64(h);
        if (h < t) {
            // claim one item, or up to kMaxClaim when a backlog has built up: the acquire
            // below is a cache-wide operation of the XCD's L2 (an invalidate), and under
            // load claims, not the hashing, bound the items per second
            const uint64_t backlog = t - h;
            uint64_t take = backlog >= 32u * kMaxClaim ? kMaxClaim : (backlog >= 64u ? backlog / 32u : 1u);
            if (take > 1) {
                // only as many items as fit kServeClaimBlocks (the first always): their
                // `blocks`, read before the claim's acquire, are a hint -- a stale value
                // changes how many items this wave takes, never what it computes
                uint32_t w = 0;
                if (lane < take)
                    w = min(__hip_atomic_load(&R.d_items[(h + lane) & mask].blocks, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT),
                            1u << 20);
                for (int d = 1; d < 64; d <<= 1) {  // inclusive prefix sum over the lanes
                    const uint32_t o = __shfl_up(w, d);
                    if (lane >= uint32_t(d)) w += o;
                }
                const uint64_t over = __ballot(lane > 0 && lane < take && w > kServeClaimBlocks);
                if (over) take = uint64_t(__builtin_ctzll(over));
            }
            uint32_t won = 0;
            if (lane == 0)
                won = __hip_atomic_compare_exchange_strong(R.d_head, &h, h + take, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT)
                          ? 1u
                          : 0u;
            if (!__builtin_amdgcn_readfirstlane(won)) continue;  // another wave moved the head
            // see the message slots the host wrote and the payload the copy engine wrote
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
            for (uint64_t k = 0; k < take; ++k) {
                const ServeItem it = R.d_items[(h + k) & mask];
                serve_item(R, it, lane, digest_lds[threadIdx.x / 64u], sched_lds[threadIdx.x / 64u]);
            }
            // digests visible to the host before the items' done flags: they were stored
            // write-through (serve_item), so it is enough that every store has completed
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            if (lane < take)
                __hip_atomic_store(R.done + ((h + lane) & mask), uint32_t(h + lane + 1), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
            last = now_ticks();
            continue;
        }
        const uint64_t now = now_ticks();
        if (now - last > 2 * R.idle_ticks || now - t0 > R.max_ticks) break;  // bounded even without the dispatcher
        __builtin_amdgcn_s_sleep(64);
    }
}

hipError_t launch_serve(const ServeRings &rings, uint32_t gen, int workgroups, hipStream_t stream)
{
    if (workgroups < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_serve, dim3(uint32_t(workgroups)), dim3(kServeThreads), 0, stream, rings, gen);
    return hipGetLastError();
}

}  // namespace hb
