// hb_plan.hip -- batched form: on-device bucketing by (algorithm, block count), work items
// of one wave each ordered longest first, and one persistent fused launch whose waves pull
// items from an atomic queue.  The pipeline is captured once in a hipGraph and replayed;
// per-run pointers reach the captured kernels through a device-side parameter block that
// a small kernel, launched ahead of the graph, fills from its own launch arguments.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hb.h"
#include "hb_device.hpp"
#include "hb_internal.hpp"
#include "hb_long.hpp"
#include "hb_plan_rules.hpp"

namespace hb {

// ---------------------------------------------------------------------------------------
// Layout constants
// ---------------------------------------------------------------------------------------

constexpr uint32_t kLdsKeys = 1024;    // keys below this are counted in LDS first
constexpr uint32_t kInvalid = 0xffffffffu;
constexpr int kThreads = 256;          // 4 waves per workgroup
constexpr int kScanThreads = 1024;
constexpr int kMaxMpl = 4;             // messages per lane per work item, at most

// VALU ops per 64-byte block of each algorithm (the compression plus word loads), used to
// weigh work items of different algorithms against each other.
__host__ __device__ constexpr uint32_t algo_cost(int a) { return a == 0 ? 340u : (a == 1 ? 620u : 1350u); }

// Run parameters, written on the device before each run (see k_set_desc).
struct PlanDesc {
    const uint8_t *algos;     // per-message ids, or nullptr
    const uint8_t *msgs;
    const uint64_t *offs;
    const uint64_t *lens;
    uint8_t *out;
    uint64_t n;
    uint32_t stride;
    int32_t algo;             // used when algos == nullptr
    int32_t sort;             // 0: one key per algorithm (index order within it)
    int32_t mpl;              // messages per lane per item
    uint32_t long_min_key;    // messages with key >= this run as long chains (0: off)
    uint32_t bulk_margin;     // bulk sized to finish in 1/bulk_margin of the longest chain (0: no limit)
};

// Meta block (device): segment bookkeeping filled by k_scan / k_items.
struct PlanMeta {
    uint32_t count[3];        // messages per algorithm
    uint32_t seg_pos[4];      // first sorted position of each algorithm's segment (+ end)
    uint32_t seg_item[4];     // first item of each segment (+ total)
    uint32_t queue;           // next item to hand out
    uint32_t pad;
    unsigned long long total_cost;
    uint32_t long_n[3];       // long-chain messages per algorithm (a prefix of its segment)
    uint32_t long_first[4];   // first long-lane index of each algorithm (padded to 64 lanes)
    uint32_t long_blocks;     // scratch wave-blocks in use
    uint32_t max_key;         // largest key present (scans stop there)
    uint32_t direct_n[3];     // long messages beyond the scratch, run as direct chains (they
                              // follow the long_n scheduled ones in the segment)
    uint32_t direct_first[4]; // first direct-lane index of each algorithm (padded to 64 lanes)
    uint32_t bulk_waves;      // persistent-kernel waves that take items (the others exit)
    unsigned long long max_chain;  // longest chain in the batch: block count x ops per block
};

// Device workspace (pointers fixed for the plan's life).
struct PlanWs {
    PlanDesc *desc;
    PlanMeta *meta;
    uint32_t *hist;           // 3 * kBins counts
    uint32_t *cursor;         // 3 * kBins running positions
    uint32_t *bin_start;      // 3 * kBins first sorted position of each key
    uint32_t *sorted;         // message indices, per-algorithm segments, padded to items
    uint32_t *order;          // item ids, longest first
    uint32_t *wave_base;      // per long-chain wave: first wave-block of its scratch region
    uint32_t *sched;          // scratch: kWaveBlockWords words per wave-block
    uint32_t sched_blocks;    // scratch capacity in wave-blocks
    uint32_t max_long_waves;  // capacity of wave_base (one more entry holds the end)
    uint32_t max_direct_waves;  // direct-chain waves at most (one per SIMD)
    uint64_t max_n;
};

// Long chains are scheduled in this algorithm order (most work per block first) when the
// scratch cannot hold all of them: slot 0 = SM3, 1 = SHA-1, 2 = MD5.
__host__ __device__ constexpr int long_order(int o) { return o == 0 ? SM3 : (o == 1 ? SHA1 : MD5); }

__device__ __forceinline__ uint32_t msg_key(uint64_t len, int sort) { return sort ? sort_key(len) : 0u; }

__device__ __forceinline__ int msg_algo(const PlanDesc &d, uint64_t i)
{
    return d.algos ? int(d.algos[i]) : d.algo;
}

__device__ __forceinline__ uint64_t lane_mask_lt()
{
    const uint32_t lane = __lane_id();
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

constexpr uint64_t kMinBulkWaves = 256;  // the persistent kernel keeps at least this many

// ---------------------------------------------------------------------------------------
// Pipeline kernels
// ---------------------------------------------------------------------------------------

__global__ void k_set_desc(PlanDesc d, PlanDesc *dst) { *dst = d; }

// Clear counts, cursors and the queue (a kernel, so the graph holds no memset node).
__global__ __launch_bounds__(kThreads) void k_zero(PlanWs ws)
{
    const uint32_t t = blockIdx.x * kThreads + threadIdx.x, step = gridDim.x * kThreads;
    for (uint32_t i = t; i < 3 * kBins; i += step) { ws.hist[i] = 0; ws.cursor[i] = 0; }
    if (t == 0) {
        PlanMeta *m = ws.meta;
        for (int a = 0; a < 3; ++a) {
            m->count[a] = 0; m->long_n[a] = 0; m->long_first[a] = 0;
            m->direct_n[a] = 0; m->direct_first[a] = 0;
        }
        m->long_first[3] = 0;
        m->direct_first[3] = 0;
        m->bulk_waves = 0xffffffffu;
        m->long_blocks = 0;
        m->max_key = 0;
        m->max_chain = 0;
        m->queue = 0;
        m->total_cost = 0;
    }
}

// Histogram of keys per algorithm.  Invalid ids are not counted (their slot is zeroed by
// k_zero_invalid).  Wave-uniform keys take one LDS atomic per wave.
__global__ __launch_bounds__(kThreads) void k_hist(PlanWs ws)
{
    __shared__ uint32_t lh[3 * kLdsKeys];
    __shared__ uint32_t lmax;
    __shared__ unsigned long long lchain;
    const PlanDesc d = *ws.desc;
    for (uint32_t i = threadIdx.x; i < 3 * kLdsKeys; i += kThreads) lh[i] = 0;
    if (threadIdx.x == 0) { lmax = 0; lchain = 0; }
    uint32_t my_max = 0;
    unsigned long long my_chain = 0;
    __syncthreads();
    const uint64_t step = uint64_t(gridDim.x) * kThreads;
    for (uint64_t base = uint64_t(blockIdx.x) * kThreads; base < d.n; base += step) {
        const uint64_t i = base + threadIdx.x;
        if (i < d.n) {
            const int a = msg_algo(d, i);
            if (a >= 0 && a < 3) {
                const uint64_t len = d.lens[i];
                const uint32_t key = msg_key(len, d.sort);
                my_max = key > my_max ? key : my_max;
                const unsigned long long chain = block_count(len) * algo_cost(a);
                my_chain = chain > my_chain ? chain : my_chain;
                const uint32_t slot = uint32_t(a) * kBins + key;
                const uint32_t first = __builtin_amdgcn_readfirstlane(slot);
                const uint64_t same = __ballot(slot == first);
                const uint64_t active = __ballot(1);
                if (same == active && key < kLdsKeys) {
                    if ((active & lane_mask_lt()) == 0)
                        atomicAdd(&lh[uint32_t(a) * kLdsKeys + key], uint32_t(__popcll(active)));
                } else if (key < kLdsKeys) {
                    atomicAdd(&lh[uint32_t(a) * kLdsKeys + key], 1u);
                } else {
                    atomicAdd(&ws.hist[slot], 1u);
                }
            }
        }
    }
    if (my_max) atomicMax(&lmax, my_max);
    if (my_chain) atomicMax(&lchain, my_chain);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < 3 * kLdsKeys; i += kThreads) {
        const uint32_t c = lh[i];
        if (c) atomicAdd(&ws.hist[(i / kLdsKeys) * kBins + (i % kLdsKeys)], c);
    }
    if (threadIdx.x == 0 && lmax) atomicMax(&ws.meta->max_key, lmax);
    if (threadIdx.x == 0 && lchain) atomicMax(&ws.meta->max_chain, lchain);
}

// Exclusive scan, longest key first within each algorithm; segments padded to whole
// items (64 * mpl positions) whose padding slots hold kInvalid.
__global__ __launch_bounds__(kScanThreads) void k_scan(PlanWs ws)
{
    __shared__ uint32_t part[kScanThreads];
    __shared__ uint32_t seg_base;
    const PlanDesc d = *ws.desc;
    const uint32_t per_item = 64u * uint32_t(d.mpl);
    const uint32_t top = ws.meta->max_key;        // keys above it are empty
    const uint32_t nkeys = top + 1;
    const uint32_t kPer = (nkeys + kScanThreads - 1) / kScanThreads;
    if (threadIdx.x == 0) seg_base = 0;
    __syncthreads();
    for (int a = 0; a < 3; ++a) {
        // thread t owns reversed keys [t*kPer, (t+1)*kPer): key = top - r
        uint32_t local = 0;
        for (uint32_t k = 0; k < kPer; ++k) {
            const uint32_t r = threadIdx.x * kPer + k;
            if (r < nkeys) local += ws.hist[a * kBins + (top - r)];
        }
        part[threadIdx.x] = local;
        __syncthreads();
        for (uint32_t off = 1; off < kScanThreads; off <<= 1) {  // inclusive Hillis-Steele
            const uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
            __syncthreads();
            part[threadIdx.x] += v;
            __syncthreads();
        }
        const uint32_t total = part[kScanThreads - 1];
        uint32_t run = seg_base + part[threadIdx.x] - local;
        for (uint32_t k = 0; k < kPer; ++k) {
            const uint32_t r = threadIdx.x * kPer + k;
            if (r < nkeys) {
                const uint32_t key = top - r;
                ws.bin_start[a * kBins + key] = run;
                run += ws.hist[a * kBins + key];
            }
        }
        const uint32_t padded = (total + per_item - 1) / per_item * per_item;
        for (uint32_t p = total + threadIdx.x; p < padded; p += kScanThreads) ws.sorted[seg_base + p] = kInvalid;
        __syncthreads();
        if (threadIdx.x == 0) {
            PlanMeta *m = ws.meta;
            m->count[a] = total;
            m->seg_pos[a] = seg_base;
            m->seg_item[a] = (a == 0 ? 0u : m->seg_item[a - 1] + (m->seg_pos[a] - m->seg_pos[a - 1]) / per_item);
            seg_base += padded;
            if (a == 2) {
                m->seg_pos[3] = seg_base;
                m->seg_item[3] = m->seg_item[2] + padded / per_item;
            }
        }
        __syncthreads();
    }
}

// Scatter message indices to their sorted positions.  Each pass handles kThreads * kR
// messages: local ranks come from LDS atomics, then one global atomic per non-empty key
// reserves the workgroup's range.
constexpr int kR = 8;
__global__ __launch_bounds__(kThreads) void k_scatter(PlanWs ws)
{
    __shared__ uint32_t lc[3 * kLdsKeys];
    const PlanDesc d = *ws.desc;
    const uint64_t chunk = uint64_t(kThreads) * kR;
    for (uint64_t base = uint64_t(blockIdx.x) * chunk; base < d.n; base += uint64_t(gridDim.x) * chunk) {
        for (uint32_t i = threadIdx.x; i < 3 * kLdsKeys; i += kThreads) lc[i] = 0;
        __syncthreads();
        uint32_t slot[kR], rank[kR];
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const uint64_t i = base + uint64_t(r) * kThreads + threadIdx.x;
            slot[r] = kInvalid;
            rank[r] = 0;
            if (i < d.n) {
                const int a = msg_algo(d, i);
                if (a >= 0 && a < 3) {
                    const uint32_t key = msg_key(d.lens[i], d.sort);
                    slot[r] = uint32_t(a) * kBins + key;
                    if (key < kLdsKeys) {
                        const uint32_t ls = uint32_t(a) * kLdsKeys + key;
                        const uint32_t first = __builtin_amdgcn_readfirstlane(ls);
                        const uint64_t same = __ballot(ls == first);
                        const uint64_t active = __ballot(1);
                        if (same == active) {
                            uint32_t b = 0;
                            if ((active & lane_mask_lt()) == 0) b = atomicAdd(&lc[ls], uint32_t(__popcll(active)));
                            b = __builtin_amdgcn_readfirstlane(b);
                            rank[r] = b + uint32_t(__popcll(active & lane_mask_lt()));
                        } else {
                            rank[r] = atomicAdd(&lc[ls], 1u);
                        }
                    } else {
                        rank[r] = ws.bin_start[slot[r]] + atomicAdd(&ws.cursor[slot[r]], 1u);
                    }
                }
            }
        }
        __syncthreads();
        // reserve this pass's range of each LDS key; lc[] becomes the absolute base
        for (uint32_t i = threadIdx.x; i < 3 * kLdsKeys; i += kThreads) {
            const uint32_t c = lc[i];
            if (c) {
                const uint32_t s = (i / kLdsKeys) * kBins + (i % kLdsKeys);
                lc[i] = ws.bin_start[s] + atomicAdd(&ws.cursor[s], c);
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            if (slot[r] == kInvalid) continue;
            const uint64_t i = base + uint64_t(r) * kThreads + threadIdx.x;
            const uint32_t a = slot[r] / kBins, key = slot[r] % kBins;
            const uint32_t pos = key < kLdsKeys ? lc[a * kLdsKeys + key] + rank[r] : rank[r];
            ws.sorted[pos] = uint32_t(i);
        }
        __syncthreads();
    }
}

// Estimated cost of an item: the (capped) block-count key of its first message -- the
// largest in the item -- times the algorithm's ops per block, times messages per lane.
// Keys are non-increasing along a segment, so costs are too.
__device__ __forceinline__ uint64_t item_cost(const PlanWs &ws, const PlanDesc &d, const PlanMeta &m, int a,
                                              uint32_t k)
{
    const uint32_t per_item = 64u * uint32_t(d.mpl);
    const uint32_t idx = ws.sorted[m.seg_pos[a] + k * per_item];
    const uint64_t key = idx == kInvalid ? 0 : msg_key(d.lens[idx], d.sort);
    return key * algo_cost(a) * uint64_t(d.mpl);
}

// Number of items of segment b that go before an item of cost c from segment a.
__device__ __forceinline__ uint32_t count_before(const PlanWs &ws, const PlanDesc &d, const PlanMeta &m, int b,
                                                 int a, uint64_t c)
{
    uint32_t lo = 0, hi = m.seg_item[b + 1] - m.seg_item[b];  // items of b, costs non-increasing
    while (lo < hi) {
        const uint32_t mid = (lo + hi) / 2;
        const uint64_t cb = item_cost(ws, d, m, b, mid);
        const bool before = cb > c || (cb == c && b < a);
        if (before) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Merge the three segments' items by cost, longest first: order[rank] = item id.
__global__ __launch_bounds__(kThreads) void k_items(PlanWs ws)
{
    const PlanDesc d = *ws.desc;
    const PlanMeta m = *ws.meta;
    const uint32_t total = m.seg_item[3];
    unsigned long long local_cost = 0;
    for (uint32_t it = blockIdx.x * kThreads + threadIdx.x; it < total; it += gridDim.x * kThreads) {
        int a = 0;
        while (a < 2 && it >= m.seg_item[a + 1]) ++a;
        const uint32_t k = it - m.seg_item[a];
        const uint64_t c = item_cost(ws, d, m, a, k);
        uint32_t rank = k;
        for (int b = 0; b < 3; ++b)
            if (b != a) rank += count_before(ws, d, m, b, a, c);
        ws.order[rank] = it;
        local_cost += c;
    }
    if (local_cost) atomicAdd(&ws.meta->total_cost, local_cost);
}

// Zero the 32-byte slots of messages whose algorithm id is unknown.
__global__ __launch_bounds__(kThreads) void k_zero_invalid(PlanWs ws)
{
    const PlanDesc d = *ws.desc;
    if (!d.algos) return;
    const uint64_t step = uint64_t(gridDim.x) * kThreads;
    for (uint64_t i = uint64_t(blockIdx.x) * kThreads + threadIdx.x; i < d.n; i += step) {
        if (d.algos[i] > SM3) {
            HB_GLOBAL uint32_t *o = reinterpret_cast<HB_GLOBAL uint32_t *>(reinterpret_cast<uintptr_t>(d.out + i * d.stride));
            for (uint32_t q = 0; q < d.stride / 4u; ++q) o[q] = 0u;
        }
    }
}

// Choose the long-chain messages: within each algorithm's segment, the leading messages
// (longest first) whose key reaches long_min_key, taken a wave (64 messages) at a time
// while the waves' scratch regions fit; a wave's region is as many wave-blocks as its
// longest message has blocks (wave_region_blocks: lane 0's count below the saturated key,
// the largest over the wave's lanes once keys saturate and the order among them is
// arbitrary).  The candidates that do not fit become direct chains (below).  One
// workgroup; each long-chain wave is algorithm-uniform.
__global__ __launch_bounds__(kScanThreads) void k_long_scan(PlanWs ws)
{
    __shared__ uint32_t part[kScanThreads];
    __shared__ unsigned long long part64[kScanThreads];
    __shared__ unsigned long long s_run;
    __shared__ uint32_t s_wave, s_stop, s_cand[3];
    const PlanDesc d = *ws.desc;
    PlanMeta *m = ws.meta;
    if (threadIdx.x == 0) { s_run = 0; s_wave = 0; }
    __syncthreads();
    for (int o = 0; o < 3; ++o) {
        const int a = long_order(o);
        uint32_t cand = 0;
        if (d.long_min_key && d.sort) {
            // messages with key >= long_min_key: a prefix of the segment
            uint32_t local = 0;
            for (uint32_t k = d.long_min_key + threadIdx.x; k <= m->max_key; k += kScanThreads)
                local += ws.hist[a * kBins + k];
            part[threadIdx.x] = local;
            __syncthreads();
            for (uint32_t off = kScanThreads / 2; off > 0; off >>= 1) {
                if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
                __syncthreads();
            }
            cand = part[0];
            __syncthreads();
        }
        const uint32_t nw = (cand + 63u) / 64u;
        const uint32_t w0 = s_wave;
        if (threadIdx.x == 0) s_stop = 0;
        __syncthreads();
        uint32_t taken = 0;
        for (uint32_t c0 = 0; c0 < nw; c0 += kScanThreads) {
            if (s_stop) break;
            const uint32_t wi = c0 + threadIdx.x;
            unsigned long long cost = 0;
            if (wi < nw) {
                const uint32_t *lane_idx = ws.sorted + m->seg_pos[a] + wi * 64u;
                // clamped to capacity + 1, which never fits, so the sums stay small
                cost = wave_region_blocks([&](uint32_t l) { return d.lens[lane_idx[l]]; },
                                          min(64u, cand - wi * 64u), uint64_t(ws.sched_blocks) + 1u);
            }
            part64[threadIdx.x] = cost;
            __syncthreads();
            for (uint32_t off = 1; off < kScanThreads; off <<= 1) {
                const unsigned long long v = threadIdx.x >= off ? part64[threadIdx.x - off] : 0ull;
                __syncthreads();
                part64[threadIdx.x] += v;
                __syncthreads();
            }
            const unsigned long long base = s_run + part64[threadIdx.x] - cost;
            const bool fits = wi < nw && base + cost <= ws.sched_blocks && w0 + wi < ws.max_long_waves;
            if (fits) ws.wave_base[w0 + wi] = uint32_t(base);
            const uint32_t nfit = uint32_t(__syncthreads_count(fits));
            __syncthreads();
            if (threadIdx.x == 0) {
                if (nfit) s_run += part64[nfit - 1];
                if (nfit < kScanThreads) s_stop = 1;
            }
            taken += nfit;
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            m->long_n[a] = min(cand, taken * 64u);
            m->long_first[a] = w0 * 64u;
            s_wave = w0 + taken;
            s_cand[a] = cand;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ws.wave_base[s_wave] = uint32_t(s_run);  // end of the last region
        m->long_first[3] = s_wave * 64u;
        m->long_blocks = uint32_t(s_run);
        // The candidates the scratch could not hold run as direct chains, each on a lane
        // of its own at the highest priority.  At most max_direct_waves waves: if more are
        // needed, only the messages whose chain cost (blocks x ops per block) reaches the
        // smallest threshold that fits are taken, across the three algorithms; the rest
        // stay with the persistent kernel.
        uint32_t left[3];
        for (int a = 0; a < 3; ++a) left[a] = s_cand[a] - m->long_n[a];
        auto chosen = [&](int a, uint64_t c) -> uint32_t {  // candidates left of cost >= c
            const uint64_t k = (c + algo_cost(a) - 1) / algo_cost(a);  // smallest key with cost >= c
            if (k > m->max_key) return 0u;
            const uint32_t key = uint32_t(k < 1 ? 1 : k);
            const uint32_t ge = ws.bin_start[a * kBins + key] + ws.hist[a * kBins + key] - m->seg_pos[a];
            return ge <= m->long_n[a] ? 0u : min(left[a], ge - m->long_n[a]);
        };
        auto waves = [&](uint64_t c) -> uint64_t {
            uint64_t w = 0;
            for (int a = 0; a < 3; ++a) w += (chosen(a, c) + 63u) / 64u;
            return w;
        };
        uint64_t c = 0;
        if (waves(0) > ws.max_direct_waves) {
            uint64_t lo = 1, hi = uint64_t(kBins) * algo_cost(SM3) + 1;  // waves(hi) == 0
            while (lo < hi) {
                const uint64_t mid = (lo + hi) / 2;
                if (waves(mid) <= ws.max_direct_waves) hi = mid;
                else lo = mid + 1;
            }
            c = lo;
        }
        uint32_t first = 0;
        for (int o = 0; o < 3; ++o) {
            const int a = long_order(o);
            const uint32_t nd = c ? chosen(a, c) : left[a];
            m->direct_n[a] = nd;
            m->direct_first[a] = first;
            first += (nd + 63u) & ~63u;
        }
        m->direct_first[3] = first;
        // When one chain is far longer than the bulk needs, the bulk runs on fewer waves:
        // enough that its items (total_cost, in the same op units as a chain) would finish in
        // 1/bulk_margin of the longest chain's time at one op per wave issue slot.  Fewer
        // bulk waves leave the long chains more issue slots and memory bandwidth.
        const bool any_cand = s_cand[0] + s_cand[1] + s_cand[2] > 0;
        const uint64_t crit = any_cand ? m->max_chain : 0;
        if (crit && d.bulk_margin) {
            const uint64_t w = (uint64_t(d.bulk_margin) * m->total_cost + crit - 1) / crit;
            m->bulk_waves = uint32_t(min<uint64_t>(max<uint64_t>(w, kMinBulkWaves), 0xffffffffull));
        }
    }
}

// Which algorithm long lane g (< long_first[3]) belongs to; i = its index in that algorithm.
__device__ __forceinline__ int long_algo(const PlanMeta &m, uint32_t g, uint32_t &i)
{
    for (int o = 0; o < 3; ++o) {
        const int a = long_order(o);
        const uint32_t end = o < 2 ? m.long_first[long_order(o + 1)] : m.long_first[3];
        if (g >= m.long_first[a] && g < end) {
            i = g - m.long_first[a];
            return a;
        }
    }
    i = 0xffffffffu;
    return MD5;
}

// Schedule words of every block of every long-chain message: one lane per (wave-block,
// lane of that wave), so each store instruction of a wave writes one contiguous KiB.
__global__ __launch_bounds__(kThreads) void k_sched(PlanWs ws)
{
    const PlanDesc d = *ws.desc;
    const PlanMeta m = *ws.meta;
    const uint32_t nwaves = m.long_first[3] / 64u;
    const uint64_t total = uint64_t(m.long_blocks) * 64u;
    for (uint64_t t = uint64_t(blockIdx.x) * kThreads + threadIdx.x; t < total; t += uint64_t(gridDim.x) * kThreads) {
        const uint32_t gb = uint32_t(t / 64u), l = uint32_t(t % 64u);
        // the wave whose region holds wave-block gb
        uint32_t lo = 0, hi = nwaves;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) / 2;
            if (ws.wave_base[mid] <= gb) lo = mid;
            else hi = mid;
        }
        uint32_t i = 0;
        const int a = long_algo(m, lo * 64u + l, i);
        if (i >= m.long_n[a]) continue;  // a padding lane
        const uint32_t idx = ws.sorted[m.seg_pos[a] + i];
        const uint64_t len = d.lens[idx];
        const uint64_t nb = block_count(len), blk = gb - ws.wave_base[lo];
        if (blk >= nb) continue;  // shorter than the wave's longest message
        uint32_t *wr = ws.sched + uint64_t(ws.wave_base[lo]) * kWaveBlockWords;
        uint32_t w[16], out[kSchedWords];
#define HB_SCHED_CASE(A)                                                                          \
        {                                                                                         \
            const Msg mm = make_msg<A>(d.msgs + d.offs[idx], len);                                \
            if (blk < len / 64u) load_full_block(mm, blk, w);                                     \
            else load_any_block<Traits<A>::kBE>(mm, blk, blk + 1 == nb, w);                       \
            sched_block<A>(w, out);                                                               \
            store_sched<A>(wr, blk, l, out);                                                      \
        }
        if (a == MD5) HB_SCHED_CASE(MD5)
        else if (a == SHA1) HB_SCHED_CASE(SHA1)
        else HB_SCHED_CASE(SM3)
#undef HB_SCHED_CASE
    }
}

// Long chains, one lane per message, at the highest wave priority; each wave's lanes are
// of one algorithm.  SCHED = 1: rounds only, from the precomputed words; SCHED = 0: the
// ordinary compression reading the message with the next block prefetched.  Waves past
// max_long_waves run the direct chains (ordinary compression) of the long messages the
// scratch could not hold, so no long chain shares the persistent kernel's issue slots at
// ordinary priority.
// One message's chain by the ordinary compression, the next block prefetched (SHA-1, SM3).
__device__ __forceinline__ void direct_chain(const PlanDesc &d, int a, uint32_t idx)
{
    const uint8_t *msg = d.msgs + d.offs[idx];
    const uint64_t len = d.lens[idx];
    uint32_t st[8];
    uint8_t *out = d.out + uint64_t(idx) * d.stride;
    if (a == MD5) { hash_message<MD5>(msg, len, st); store_digest<MD5>(out, st, d.stride); }
    else if (a == SHA1) { hash_message_prefetch<SHA1>(msg, len, st); store_digest<SHA1>(out, st, d.stride); }
    else { hash_message_prefetch<SM3>(msg, len, st); store_digest<SM3>(out, st, d.stride); }
}

template <int SCHED>
__device__ __forceinline__ void long_lane(const PlanWs &ws, uint32_t g)
{
    const PlanDesc d = *ws.desc;
    const PlanMeta m = *ws.meta;
    const uint32_t wave_first = g & ~63u;
    if (g >= ws.max_long_waves * 64u) {
        // direct chains: the long messages the scratch could not hold
        const uint32_t dg = g - ws.max_long_waves * 64u;
        if ((dg & ~63u) >= m.direct_first[3]) return;
        int a = MD5;
        for (int o = 0; o < 3; ++o) {
            const int b = long_order(o);
            const uint32_t end = o < 2 ? m.direct_first[long_order(o + 1)] : m.direct_first[3];
            if (dg >= m.direct_first[b] && dg < end) a = b;
        }
        const uint32_t i = dg - m.direct_first[a];
        if (i >= m.direct_n[a]) return;  // padding lane
        __builtin_amdgcn_s_setprio(3);
        direct_chain(d, a, ws.sorted[m.seg_pos[a] + m.long_n[a] + i]);
        __builtin_amdgcn_s_setprio(0);
        return;
    }
    if (wave_first >= m.long_first[3]) return;
    uint32_t i = 0;
    const int a = long_algo(m, wave_first, i);
    i = g - m.long_first[a];
    if (i >= m.long_n[a]) return;  // padding lane
    __builtin_amdgcn_s_setprio(3);
    const uint32_t idx = ws.sorted[m.seg_pos[a] + i];
    const uint64_t nb = block_count(d.lens[idx]);
    if constexpr (SCHED) {
        const uint32_t w = g / 64u;
        // k_long_scan sizes a region for its wave's longest message, so nb never exceeds
        // it; the check keeps any lane from reading past its region all the same
        if (nb <= uint64_t(ws.wave_base[w + 1]) - ws.wave_base[w]) {
            uint32_t st[8];
            uint8_t *out = d.out + uint64_t(idx) * d.stride;
            const uint32_t *wr = ws.sched + uint64_t(ws.wave_base[w]) * kWaveBlockWords;
            const uint32_t l = g % 64u;
            if (a == MD5) { chain_from_sched<MD5>(wr, l, nb, st); store_digest<MD5>(out, st, d.stride); }
            else if (a == SHA1) { chain_from_sched<SHA1>(wr, l, nb, st); store_digest<SHA1>(out, st, d.stride); }
            else { chain_from_sched<SM3>(wr, l, nb, st); store_digest<SM3>(out, st, d.stride); }
        } else {
            direct_chain(d, a, idx);
        }
    } else {
        direct_chain(d, a, idx);
    }
    __builtin_amdgcn_s_setprio(0);
}

template <int SCHED>
__global__ __launch_bounds__(kThreads) void k_hash_long(PlanWs ws)
{
    long_lane<SCHED>(ws, blockIdx.x * kThreads + threadIdx.x);
}

// Message-load schemes of the persistent kernel (the plan's "variant", a tuned choice):
//   0  whole blocks in bursts of the default depth (MD5 four, SHA-1 / SM3 two)
//   1  SHA-1 / SM3: one block at a time with the next block's loads in flight during the
//      current compression; MD5 as 0
//   2  one block per load (no bursts)
//   3  bursts of two blocks for every algorithm
//   4  bursts of four blocks for every algorithm
constexpr int kLoadSchemes = 5;

template <int V, int A>
constexpr int scheme_burst() { return V == 2 ? 1 : (V == 3 ? 2 : (V == 4 ? 4 : kDefaultBurst<A>)); }

template <int A, int V>
__device__ __forceinline__ void hash_lane(const PlanDesc &d, uint32_t idx)
{
    uint32_t s[8];
    const uint64_t off = reinterpret_cast<const HB_GLOBAL uint64_t *>(reinterpret_cast<uintptr_t>(d.offs))[idx];
    const uint64_t len = reinterpret_cast<const HB_GLOBAL uint64_t *>(reinterpret_cast<uintptr_t>(d.lens))[idx];
    if constexpr (V == 1 && A != MD5) hash_message_prefetch<A>(d.msgs + off, len, s);
    else hash_message<A, scheme_burst<V, A>()>(d.msgs + off, len, s);
    store_digest<A>(d.out + uint64_t(idx) * d.stride, s, d.stride);
}

// Persistent fused kernel: each wave takes items from the queue until none are left.
// An item is 64 * mpl sorted positions of one algorithm; lane l hashes positions
// l, l + 64, ... of it.  Items whose cost exceeds the average per-wave share run at raised
// wave priority so the longest chains keep their issue slots.  PF is the load scheme (see
// kLoadSchemes).
template <int PF>
__device__ __forceinline__ void persistent_wave(const PlanWs &ws, uint32_t block, uint32_t nblocks)
{
    const PlanDesc d = *ws.desc;
    const PlanMeta *mp = ws.meta;
    const uint32_t total = mp->seg_item[3];
    const uint32_t per_item = 64u * uint32_t(d.mpl);
    const uint64_t waves = uint64_t(nblocks) * (kThreads / 64);
    const uint64_t share = mp->total_cost / (waves ? waves : 1);
    const uint32_t lane = __lane_id();
    uint32_t bulk = mp->bulk_waves;
    if (bulk == 0xffffffffu && d.bulk_margin && total) {
        // no long-chain pass sized the bulk: size it from the longest item (the first in
        // the order), by the same rule
        const uint32_t item0 = ws.order[0];
        int a0 = 0;
        while (a0 < 2 && item0 >= mp->seg_item[a0 + 1]) ++a0;
        const uint64_t crit = item0 < total ? item_cost(ws, d, *mp, a0, item0 - mp->seg_item[a0]) : 0;
        if (crit) {
            const uint64_t w = (uint64_t(d.bulk_margin) * mp->total_cost + crit - 1) / crit;
            bulk = uint32_t(min<uint64_t>(max<uint64_t>(w, kMinBulkWaves), 0xffffffffull));
        }
    }
    if (block * (kThreads / 64u) + threadIdx.x / 64u >= bulk) return;  // surplus wave
    for (;;) {
        uint32_t it = 0;
        if (lane == 0) it = atomicAdd(&ws.meta->queue, 1u);
        it = __builtin_amdgcn_readfirstlane(it);
        if (it >= total) break;
        const uint32_t item = ws.order[it];
        if (item >= total) continue;  // never taken when the ranks form a permutation
        int a = 0;
        while (a < 2 && item >= mp->seg_item[a + 1]) ++a;
        const uint32_t pos0 = mp->seg_pos[a] + (item - mp->seg_item[a]) * per_item;
        const uint32_t first = ws.sorted[pos0];
        const uint64_t cost = first == kInvalid ? 0 : uint64_t(msg_key(d.lens[first], d.sort)) * algo_cost(a) * d.mpl;
        if (cost > share) __builtin_amdgcn_s_setprio(2);
        else __builtin_amdgcn_s_setprio(0);
        const uint32_t long_end = mp->seg_pos[a] + mp->long_n[a] + mp->direct_n[a];  // k_hash_long's
        if (pos0 + per_item <= long_end) continue;
        for (int j = 0; j < d.mpl; ++j) {
            const uint32_t pos = pos0 + uint32_t(j) * 64u + lane;
            if (pos < long_end) continue;
            const uint32_t idx = ws.sorted[pos];
            if (idx == kInvalid) continue;
            if (a == MD5) hash_lane<MD5, PF>(d, idx);
            else if (a == SHA1) hash_lane<SHA1, PF>(d, idx);
            else hash_lane<SM3, PF>(d, idx);
        }
    }
    __builtin_amdgcn_s_setprio(0);
}

template <int PF>
__global__ __launch_bounds__(kThreads) void k_hash_persistent(PlanWs ws)
{
    persistent_wave<PF>(ws, blockIdx.x, gridDim.x);
}

// The long-chain kernel and the persistent kernel in one launch: workgroups below
// long_blocks run the long chains (dispatched first), the rest the bulk.  Same work and
// concurrency as the two kernels on two streams, without a second stream.
template <int SCHED, int PF>
__global__ __launch_bounds__(kThreads) void k_hash_fused(PlanWs ws, uint32_t long_blocks)
{
    if (blockIdx.x < long_blocks) long_lane<SCHED>(ws, blockIdx.x * kThreads + threadIdx.x);
    else persistent_wave<PF>(ws, blockIdx.x - long_blocks, gridDim.x - long_blocks);
}

// ---------------------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------------------

struct TuneKey {
    std::string arch;
    int cus;
    int algo_mask;
    int len_bucket;
    bool operator<(const TuneKey &o) const
    {
        if (arch != o.arch) return arch < o.arch;
        if (cus != o.cus) return cus < o.cus;
        if (algo_mask != o.algo_mask) return algo_mask < o.algo_mask;
        return len_bucket < o.len_bucket;
    }
};

struct TuneChoice {
    int waves_per_cu;
    int mpl;
    int variant;
};

static std::mutex g_tune_mu;
static std::map<TuneKey, TuneChoice> g_tune_cache;
static bool g_tune_loaded = false;

// Optional persistence: HB_TUNE_CACHE names a text file of lines
// "arch cus algo_mask length_bucket waves_per_cu msgs_per_lane variant".
static void load_tune_cache()
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("HB_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char arch[64];
    int cus, mask, bucket, w, m, v;
    while (std::fscanf(f, "%63s %d %d %d %d %d %d", arch, &cus, &mask, &bucket, &w, &m, &v) == 7)
        if (w > 0 && w <= 64 && m > 0 && m <= kMaxMpl && v >= 0 && v < kLoadSchemes)
            g_tune_cache[TuneKey{arch, cus, mask, bucket}] = TuneChoice{w, m, v};
    std::fclose(f);
}

static void save_tune_cache()
{
    const char *path = std::getenv("HB_TUNE_CACHE");
    if (!path) return;
    std::lock_guard<std::mutex> g(g_tune_mu);
    FILE *f = std::fopen(path, "w");
    if (!f) return;
    for (auto &kv : g_tune_cache)
        std::fprintf(f, "%s %d %d %d %d %d %d\n", kv.first.arch.c_str(), kv.first.cus, kv.first.algo_mask,
                     kv.first.len_bucket, kv.second.waves_per_cu, kv.second.mpl, kv.second.variant);
    std::fclose(f);
}

}  // namespace hb

struct hb_plan {
    hb::PlanWs ws{};
    int flags = 0;
    int device = 0;
    int cus = 0;
    std::string arch;
    int waves_per_cu = 16;
    int mpl = 1;
    int variant = 0;
    bool tuned = false;
    int tune_bucket = -1;           // length bucket the autotuner keyed its choice by
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_mpl = 0, graph_sort = -1;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free, ev_pending;  // hash-kernel timing
    bool long_on = false;           // long-chain path enabled
    bool long_sched = true;         // precomputed schedule words (else direct reads)
    uint32_t long_min_key = 0;
    uint32_t bulk_margin = 4;     // HB_BULK_MARGIN
    hipStream_t side = nullptr;     // long-chain kernel runs here, beside the persistent kernel
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    double kernel_ms_sum = 0.0;
    int kernel_ms_count = 0;
    void *alloc = nullptr;
};

namespace hb {

static void drop_graph(hb_plan *p)
{
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

static int grid_items(const hb_plan *p) { return p->cus * 4; }

// Event pair bracketing the next hash launch (reused once collected).
static std::pair<hipEvent_t, hipEvent_t> take_events(hb_plan *p)
{
    if (!p->ev_free.empty()) {
        auto e = p->ev_free.back();
        p->ev_free.pop_back();
        return e;
    }
    std::pair<hipEvent_t, hipEvent_t> e{nullptr, nullptr};
    if (hipEventCreate(&e.first) != hipSuccess || hipEventCreate(&e.second) != hipSuccess) return {nullptr, nullptr};
    return e;
}

// Fold the durations of finished timed launches into the running average.
static void collect_timing(hb_plan *p, bool wait)
{
    std::vector<std::pair<hipEvent_t, hipEvent_t>> keep;
    for (auto &e : p->ev_pending) {
        if (!wait && hipEventQuery(e.second) != hipSuccess) { keep.push_back(e); continue; }
        float ms = 0.f;
        if (hipEventSynchronize(e.second) == hipSuccess && hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) {
            p->kernel_ms_sum += ms;
            p->kernel_ms_count += 1;
        }
        p->ev_free.push_back(e);
    }
    p->ev_pending.swap(keep);
}

template <int V>
static void launch_fused_v(bool sched, dim3 grid, hipStream_t s, const PlanWs &ws, uint32_t long_blocks)
{
    if (sched) hipLaunchKernelGGL((k_hash_fused<1, V>), grid, dim3(kThreads), 0, s, ws, long_blocks);
    else hipLaunchKernelGGL((k_hash_fused<0, V>), grid, dim3(kThreads), 0, s, ws, long_blocks);
}

static void launch_fused(bool sched, int variant, dim3 grid, hipStream_t s, const PlanWs &ws, uint32_t long_blocks)
{
    switch (variant) {
    case 1: launch_fused_v<1>(sched, grid, s, ws, long_blocks); break;
    case 2: launch_fused_v<2>(sched, grid, s, ws, long_blocks); break;
    case 3: launch_fused_v<3>(sched, grid, s, ws, long_blocks); break;
    case 4: launch_fused_v<4>(sched, grid, s, ws, long_blocks); break;
    default: launch_fused_v<0>(sched, grid, s, ws, long_blocks); break;
    }
}

static void launch_persistent(int variant, dim3 grid, hipStream_t s, const PlanWs &ws)
{
    switch (variant) {
    case 1: hipLaunchKernelGGL(k_hash_persistent<1>, grid, dim3(kThreads), 0, s, ws); break;
    case 2: hipLaunchKernelGGL(k_hash_persistent<2>, grid, dim3(kThreads), 0, s, ws); break;
    case 3: hipLaunchKernelGGL(k_hash_persistent<3>, grid, dim3(kThreads), 0, s, ws); break;
    case 4: hipLaunchKernelGGL(k_hash_persistent<4>, grid, dim3(kThreads), 0, s, ws); break;
    default: hipLaunchKernelGGL(k_hash_persistent<0>, grid, dim3(kThreads), 0, s, ws); break;
    }
}

// Enqueue the pipeline (after k_set_desc) on stream s.  With `timed`, HIP events on s
// bracket the persistent hashing kernel.
static hipError_t enqueue_pipeline(hb_plan *p, hipStream_t s, bool timed)
{
    const PlanWs &ws = p->ws;
    const int g = grid_items(p);
    hipLaunchKernelGGL(k_zero, dim3(g), dim3(kThreads), 0, s, ws);
    hipLaunchKernelGGL(k_hist, dim3(g), dim3(kThreads), 0, s, ws);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, ws);
    hipLaunchKernelGGL(k_scatter, dim3(g), dim3(kThreads), 0, s, ws);
    hipLaunchKernelGGL(k_items, dim3(g), dim3(kThreads), 0, s, ws);
    hipLaunchKernelGGL(k_zero_invalid, dim3(g), dim3(kThreads), 0, s, ws);
    const int hash_blocks = (p->cus * p->waves_per_cu + 3) / 4;
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (timed) ev = take_events(p);
    if (p->long_on) {
        hipLaunchKernelGGL(k_long_scan, dim3(1), dim3(kScanThreads), 0, s, ws);
        if (p->long_sched) hipLaunchKernelGGL(k_sched, dim3(g), dim3(kThreads), 0, s, ws);
    }
    if (ev.first) hipEventRecord(ev.first, s);
    const bool fused = p->long_on && !p->side;
    if (fused) {
        // no side stream: long chains and bulk in one launch, the chains' workgroups first
        const uint32_t long_blocks =
            uint32_t((uint64_t(ws.max_long_waves + ws.max_direct_waves) * 64u + kThreads - 1) / kThreads);
        const dim3 grid{long_blocks + uint32_t(hash_blocks), 1, 1};
        launch_fused(p->long_sched, p->variant, grid, s, ws, long_blocks);
    } else if (p->long_on) {
        // fork: the long chains start first on the side stream and run beside the bulk.  A
        // failed fork or join is returned: unjoined, the run's stream could report the
        // digests done before the long chains wrote theirs.
        hipError_t fe = hipEventRecord(p->ev_fork, s);
        if (fe == hipSuccess) fe = hipStreamWaitEvent(p->side, p->ev_fork, 0);
        if (fe != hipSuccess) return fe;
        const int long_blocks =
            int((uint64_t(ws.max_long_waves + ws.max_direct_waves) * 64u + kThreads - 1) / kThreads);
        if (p->long_sched) hipLaunchKernelGGL(k_hash_long<1>, dim3(long_blocks), dim3(kThreads), 0, p->side, ws);
        else hipLaunchKernelGGL(k_hash_long<0>, dim3(long_blocks), dim3(kThreads), 0, p->side, ws);
        if ((fe = hipGetLastError()) != hipSuccess) return fe;
        if ((fe = hipEventRecord(p->ev_join, p->side)) != hipSuccess) return fe;
    }
    if (!fused) {
        launch_persistent(p->variant, dim3(hash_blocks), s, ws);
    }
    if (p->long_on && !fused) {  // join
        const hipError_t je = hipStreamWaitEvent(s, p->ev_join, 0);
        if (je != hipSuccess) return je;
    }
    if (ev.first) {
        hipEventRecord(ev.second, s);
        p->ev_pending.push_back(ev);
        if (p->ev_pending.size() > 64) collect_timing(p, false);
    }
    return hipGetLastError();
}

static int launch_run(hb_plan *p, const PlanDesc &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_desc, dim3(1), dim3(1), 0, s, d, p->ws.desc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "hb_plan_run: parameter kernel");
    const bool use_graph = (p->flags & HB_PLAN_GRAPH) != 0;
    if (use_graph) {
        if (p->exec && (p->graph_mpl != d.mpl || p->graph_sort != d.sort)) drop_graph(p);
        if (!p->exec) {
            e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_error(e, "hb_plan_run: begin capture");
            hipError_t le = enqueue_pipeline(p, p->cap_stream, false);
            e = hipStreamEndCapture(p->cap_stream, &p->graph);
            if (le != hipSuccess) { drop_graph(p); return hip_error(le, "hb_plan_run: captured launch"); }
            if (e != hipSuccess) { drop_graph(p); return hip_error(e, "hb_plan_run: end capture"); }
            e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) { drop_graph(p); return hip_error(e, "hb_plan_run: instantiate"); }
            p->graph_mpl = d.mpl;
            p->graph_sort = d.sort;
        }
        e = hipGraphLaunch(p->exec, s);
        if (e != hipSuccess) return hip_error(e, "hb_plan_run: graph launch");
        return HB_OK;
    }
    e = enqueue_pipeline(p, s, true);
    if (e != hipSuccess) return hip_error(e, "hb_plan_run: launch");
    return HB_OK;
}

// Length bucket of a batch, from the plan's own histogram of (algorithm, block count)
// after a run: 16 x floor(log2(mean blocks per message)) + floor(log2(longest / mean)),
// capped at 15.  Batches of equal mean length but very different spread (fixed lengths,
// uniform, log-normal) land in different buckets.
static int length_bucket(const hb_plan *p, hipStream_t s, int &bucket)
{
    std::vector<uint32_t> hist(3ull * kBins);
    PlanMeta meta{};
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemcpy(hist.data(), p->ws.hist, hist.size() * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&meta, p->ws.meta, sizeof(meta), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_error(e, "hb_plan_run: autotune length bucket");
    uint64_t count = 0, blocks = 0;
    for (uint64_t k = 0; k < hist.size(); ++k) {
        count += hist[k];
        blocks += uint64_t(hist[k]) * (k % kBins);
    }
    const uint64_t mean = count ? std::max<uint64_t>(1, blocks / count) : 1;
    const uint64_t longest = std::max<uint64_t>(meta.max_key, 1);
    auto ilog2 = [](uint64_t x) { int r = 0; while (x > 1) { x >>= 1; ++r; } return r; };
    bucket = 16 * ilog2(mean) + std::min(15, ilog2(longest / mean));
    return HB_OK;
}

// Time each launch choice on this run's input and keep the fastest, cached per device,
// algorithm mix and length bucket: waves per CU, messages per lane and the message-load
// scheme (bursts of 1, 2 or 4 whole blocks, or next-block prefetch; kLoadSchemes).
static int autotune(hb_plan *p, const PlanDesc &d0, hipStream_t s, int algo_mask)
{
    const int flags_saved = p->flags;
    p->flags &= ~HB_PLAN_GRAPH;
    // one run with the current choice fills the histogram that names the length bucket
    PlanDesc d = d0;
    d.mpl = p->mpl;
    int rc = launch_run(p, d, s);
    TuneKey key{p->arch, p->cus, algo_mask, 0};
    if (rc == HB_OK) rc = length_bucket(p, s, key.len_bucket);
    if (rc != HB_OK) { p->flags = flags_saved; return rc; }
    load_tune_cache();
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            p->waves_per_cu = it->second.waves_per_cu;
            p->mpl = it->second.mpl;
            p->variant = it->second.variant;
            p->flags = flags_saved;
            p->tune_bucket = key.len_bucket;
            return HB_OK;
        }
    }
    float best = 1e30f;
    TuneChoice bestc{p->waves_per_cu, p->mpl, p->variant};
    const int wpcs[] = {8, 16, 32};
    const int mpls[] = {1, 2};
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e != hipSuccess) { p->flags = flags_saved; return hip_error(e, "hb_plan_run: autotune events"); }
    for (int var = 0; var < kLoadSchemes && rc == HB_OK; ++var)
        for (int mpl : mpls)
            for (int w : wpcs) {
                p->waves_per_cu = w;
                p->variant = var;
                p->mpl = mpl;
                d.mpl = mpl;
                float tot = 0.f;
                for (int rep = 0; rep < 2 && rc == HB_OK; ++rep) {
                    hipEventRecord(a, s);
                    rc = launch_run(p, d, s);
                    hipEventRecord(b, s);
                    hipEventSynchronize(b);
                    float ms = 0.f;
                    hipEventElapsedTime(&ms, a, b);
                    if (rep) tot += ms;  // first repetition is a warm-up
                }
                if (rc == HB_OK && tot < best) { best = tot; bestc = TuneChoice{w, mpl, var}; }
            }
    hipEventDestroy(a);
    hipEventDestroy(b);
    collect_timing(p, true);
    p->kernel_ms_sum = 0.0;
    p->kernel_ms_count = 0;
    p->flags = flags_saved;
    p->waves_per_cu = bestc.waves_per_cu;
    p->mpl = bestc.mpl;
    p->variant = bestc.variant;
    p->tune_bucket = key.len_bucket;
    if (rc != HB_OK) return rc;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune_cache[key] = bestc;
    }
    save_tune_cache();
    return HB_OK;
}

// ---------------------------------------------------------------------------------------
// Allocation-free batched run: the plan's pipeline on a workspace that lives in a static
// device array, for callers that cannot allocate (code under graph capture, serving loops
// that must not call the allocator).  Long chains run as direct chains beside the bulk in
// one launch (no schedule scratch), at most kStaticMaxN messages per call.
// ---------------------------------------------------------------------------------------

constexpr uint64_t kStaticMaxN = 1ull << 20;
constexpr uint64_t kStaticLongWaves = 3;  // no scheduled long waves: wave_base holds only the end
constexpr uint64_t up256(uint64_t x) { return (x + 255) & ~uint64_t(255); }
constexpr uint64_t kStaticDesc = up256(sizeof(PlanDesc)), kStaticMeta = up256(sizeof(PlanMeta));
constexpr uint64_t kStaticBins = up256(3ull * kBins * 4);
constexpr uint64_t kStaticSorted = up256((kStaticMaxN + 3ull * 64 * kMaxMpl) * 4);
constexpr uint64_t kStaticOrder = up256((kStaticMaxN / 64 + 4) * 4);
constexpr uint64_t kStaticWaveBase = up256((kStaticLongWaves + 1) * 4);
constexpr uint64_t kStaticBytes =
    kStaticDesc + kStaticMeta + 3 * kStaticBins + kStaticSorted + kStaticOrder + kStaticWaveBase;

// The workspace: one copy per device, held until the process ends.  Host code never uses
// this name as an address (on the host it is only a handle); it uses the device address
// that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint8_t scratch[kStaticBytes];

constexpr int kStaticDevices = 64;

struct StaticDevice {
    std::once_flag once;
    int status = HB_OK;
    std::string why;
    uint8_t *ptr = nullptr;  // device address of `scratch` on this device
    int cus = 0;
};

static StaticDevice g_static[kStaticDevices];

// Set-up on the first call on a device, with that device current: the array's address
// and the CU count (hipGetSymbolAddress and an attribute query; nothing is allocated).
static StaticDevice *static_device(int dev)
{
    if (dev < 0 || dev >= kStaticDevices) return nullptr;
    StaticDevice *sd = &g_static[dev];
    std::call_once(sd->once, [sd, dev] {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            sd->status = HB_EHIP;
            sd->why = std::string("hash_batch_bucketed_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e);
            return;
        }
        int cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess || cus <= 0) {
            sd->status = HB_EHIP;
            sd->why = std::string("hash_batch_bucketed_noalloc: CU count: ") + hipGetErrorString(e);
            return;
        }
        sd->ptr = static_cast<uint8_t *>(ptr);
        sd->cus = cus;
    });
    return sd;
}

// The plan workspace carved out of the device's copy of the array.
static PlanWs static_ws(uint8_t *base, int cus)
{
    PlanWs ws{};
    uint8_t *c = base;
    ws.desc = reinterpret_cast<PlanDesc *>(c); c += kStaticDesc;
    ws.meta = reinterpret_cast<PlanMeta *>(c); c += kStaticMeta;
    ws.hist = reinterpret_cast<uint32_t *>(c); c += kStaticBins;
    ws.cursor = reinterpret_cast<uint32_t *>(c); c += kStaticBins;
    ws.bin_start = reinterpret_cast<uint32_t *>(c); c += kStaticBins;
    ws.sorted = reinterpret_cast<uint32_t *>(c); c += kStaticSorted;
    ws.order = reinterpret_cast<uint32_t *>(c); c += kStaticOrder;
    ws.wave_base = reinterpret_cast<uint32_t *>(c);
    ws.sched = nullptr;  // no schedule scratch: every long chain is a direct chain
    ws.sched_blocks = 0;
    ws.max_long_waves = uint32_t(kStaticLongWaves);
    ws.max_direct_waves = uint32_t(cus) * 4u;
    ws.max_n = kStaticMaxN;
    return ws;
}

}  // namespace hb

using namespace hb;

extern "C" {

int hb_plan_create(hb_plan **plan, uint64_t max_n, int flags)
{
    if (!plan) return set_error(HB_EINVAL, "hb_plan_create: null plan pointer");
    *plan = nullptr;
    if (max_n == 0 || max_n > (1ull << 31))
        return set_error(HB_EINVAL, "hb_plan_create: max_n must be in [1, 2^31]");
    hb_plan *p = new hb_plan();
    p->flags = flags;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { delete p; return hip_error(e, "hb_plan_create: hipGetDevice"); }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, p->device);
    if (e != hipSuccess) { delete p; return hip_error(e, "hb_plan_create: properties"); }
    p->cus = prop.multiProcessorCount;
    p->arch = prop.gcnArchName;
    const uint64_t items_cap = max_n / 64 + 4;
    const uint64_t sorted_cap = max_n + 3ull * 64 * kMaxMpl;
    auto up = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
    const uint64_t sz_desc = up(sizeof(PlanDesc)), sz_meta = up(sizeof(PlanMeta));
    const uint64_t sz_bins = up(3ull * kBins * 4);
    const uint64_t sz_sorted = up(sorted_cap * 4), sz_order = up(items_cap * 4);
    // long-chain scratch: HB_LONG_SCRATCH_MB (default 1024) of precomputed block words for
    // messages of at least HB_LONG_MIN_BLOCKS (default 256) blocks
    p->long_on = !(flags & HB_PLAN_NO_LONG) && !(flags & HB_PLAN_NO_SORT);
    uint64_t scratch_mb = 1024, min_blocks = 256;
    if (const char *v = std::getenv("HB_LONG_SCRATCH_MB")) scratch_mb = std::strtoull(v, nullptr, 10);
    if (const char *v = std::getenv("HB_LONG_MIN_BLOCKS")) min_blocks = std::strtoull(v, nullptr, 10);
    if (scratch_mb == 0 || min_blocks < 2 || min_blocks >= kBins) p->long_on = false;
    if (const char *v = std::getenv("HB_LONG_MODE")) p->long_sched = std::strcmp(v, "direct") != 0;
    if (const char *v = std::getenv("HB_BULK_MARGIN")) p->bulk_margin = uint32_t(std::strtoul(v, nullptr, 10));
    uint64_t sched_blocks = 0, long_waves = 0, scratch_blocks = 0;
    if (p->long_on) {
        // wave-blocks of scratch; direct mode allocates none (the budget then only bounds
        // how many waves run as long chains)
        sched_blocks = std::min<uint64_t>(scratch_mb * (1ull << 20) / (kWaveBlockWords * 4), 0xffffffffull);
        long_waves = std::min<uint64_t>(sched_blocks / min_blocks + 3, 1ull << 24);
        scratch_blocks = p->long_sched ? sched_blocks : 0;
        p->long_min_key = uint32_t(min_blocks);
    }
    const uint64_t sz_long = up((long_waves + 1) * 4), sz_sched = up(scratch_blocks * kWaveBlockWords * 4);
    const uint64_t total = sz_desc + sz_meta + 3 * sz_bins + sz_sorted + sz_order + sz_long + sz_sched;
    e = hipMalloc(&p->alloc, total);
    if (e != hipSuccess) { delete p; return set_error(HB_ENOMEM, "hb_plan_create: workspace allocation failed"); }
    char *c = static_cast<char *>(p->alloc);
    p->ws.desc = reinterpret_cast<PlanDesc *>(c); c += sz_desc;
    p->ws.meta = reinterpret_cast<PlanMeta *>(c); c += sz_meta;
    p->ws.hist = reinterpret_cast<uint32_t *>(c); c += sz_bins;
    p->ws.cursor = reinterpret_cast<uint32_t *>(c); c += sz_bins;
    p->ws.bin_start = reinterpret_cast<uint32_t *>(c); c += sz_bins;
    p->ws.sorted = reinterpret_cast<uint32_t *>(c); c += sz_sorted;
    p->ws.order = reinterpret_cast<uint32_t *>(c); c += sz_order;
    p->ws.wave_base = reinterpret_cast<uint32_t *>(c); c += sz_long;
    p->ws.sched = reinterpret_cast<uint32_t *>(c);
    p->ws.sched_blocks = uint32_t(sched_blocks);
    p->ws.max_long_waves = uint32_t(long_waves);
    p->ws.max_direct_waves = p->long_on ? uint32_t(p->cus) * 4u : 0u;
    p->ws.max_n = max_n;
    // Streams only where needed: each stream may take one of the process's few hardware
    // queues, and streams sharing a queue wait behind each other's kernels.
    e = hipSuccess;
    if (flags & HB_PLAN_GRAPH) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess && p->long_on && !(flags & HB_PLAN_LONG_INLINE)) {
        if ((e = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking)) == hipSuccess &&
            (e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming)) == hipSuccess)
            e = hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        hb_plan_destroy(p);
        return hip_error(e, "hb_plan_create: stream/event");
    }
    if (const char *w = std::getenv("HB_WAVES_PER_CU")) p->waves_per_cu = std::atoi(w) > 0 ? std::atoi(w) : 16;
    *plan = p;
    return HB_OK;
}

int hb_plan_run(hb_plan *p, const uint8_t *algos, int algo, const uint8_t *messages, const uint64_t *offsets,
                const uint64_t *lengths, uint64_t n, uint8_t *digests_out, void *stream)
{
    if (!p) return set_error(HB_EINVAL, "hb_plan_run: null plan");
    if (!algos && digest_size(algo) == 0) return set_error(HB_EINVAL, "hb_plan_run: unknown algorithm id");
    if (n == 0) return HB_OK;
    if (n > p->ws.max_n) return set_error(HB_EINVAL, "hb_plan_run: n exceeds the plan's max_n");
    if (!messages || !offsets || !lengths || !digests_out)
        return set_error(HB_EINVAL, "hb_plan_run: null device pointer");
    if (reinterpret_cast<uintptr_t>(digests_out) & 3u)
        return set_error(HB_EINVAL, "hb_plan_run: digests_out must be 4-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    PlanDesc d{};
    d.algos = algos;
    d.msgs = messages;
    d.offs = offsets;
    d.lens = lengths;
    d.out = digests_out;
    d.n = n;
    d.stride = algos ? 32u : uint32_t(digest_size(algo));
    d.algo = algos ? 0 : algo;
    d.sort = (p->flags & HB_PLAN_NO_SORT) ? 0 : 1;
    d.long_min_key = (p->long_on && d.sort) ? p->long_min_key : 0;
    d.bulk_margin = p->bulk_margin;
    if ((p->flags & HB_PLAN_AUTOTUNE) && !p->tuned) {
        d.mpl = p->mpl;
        const int mask = algos ? 7 : (1 << algo);
        int rc = autotune(p, d, s, mask);
        if (rc != HB_OK) return rc;
        p->tuned = true;
    }
    d.mpl = p->mpl;
    return launch_run(p, d, s);
}

int hb_plan_config(const hb_plan *p, int *waves_per_cu, int *msgs_per_lane, int *variant)
{
    if (!p) return set_error(HB_EINVAL, "hb_plan_config: null plan");
    if (waves_per_cu) *waves_per_cu = p->waves_per_cu;
    if (msgs_per_lane) *msgs_per_lane = p->mpl;
    if (variant) *variant = p->variant;
    return HB_OK;
}

int hb_plan_set_config(hb_plan *p, int waves_per_cu, int msgs_per_lane, int variant)
{
    if (!p) return set_error(HB_EINVAL, "hb_plan_set_config: null plan");
    if (waves_per_cu < 0 || waves_per_cu > 64 || msgs_per_lane < 0 || msgs_per_lane > kMaxMpl || variant < 0 ||
        variant >= kLoadSchemes)
        return set_error(HB_EINVAL, "hb_plan_set_config: out of range");
    if (waves_per_cu) p->waves_per_cu = waves_per_cu;
    if (msgs_per_lane) p->mpl = msgs_per_lane;
    p->variant = variant;
    p->tuned = true;
    drop_graph(p);
    return HB_OK;
}

double hb_plan_kernel_ms(hb_plan *p)
{
    if (!p) return -1.0;
    collect_timing(p, true);
    if (p->kernel_ms_count == 0) return -1.0;
    const double r = p->kernel_ms_sum / p->kernel_ms_count;
    p->kernel_ms_sum = 0.0;
    p->kernel_ms_count = 0;
    return r;
}

void hb_plan_destroy(hb_plan *p)
{
    if (!p) return;
    if (p->cap_stream) hipStreamSynchronize(p->cap_stream);
    hipDeviceSynchronize();
    drop_graph(p);
    collect_timing(p, true);
    for (auto &e : p->ev_free) { hipEventDestroy(e.first); hipEventDestroy(e.second); }
    if (p->cap_stream) hipStreamDestroy(p->cap_stream);
    if (p->side) hipStreamDestroy(p->side);
    if (p->ev_fork) hipEventDestroy(p->ev_fork);
    if (p->ev_join) hipEventDestroy(p->ev_join);
    if (p->alloc) hipFree(p->alloc);
    delete p;
}

int hash_batch_bucketed_noalloc(const uint8_t *algos, int algo, const uint8_t *messages, const uint64_t *offsets,
                                const uint64_t *lengths, uint64_t n, uint8_t *digests_out, void *stream)
{
    if (!algos && digest_size(algo) == 0) return set_error(HB_EINVAL, "hash_batch_bucketed_noalloc: unknown algorithm id");
    if (n == 0) return HB_OK;
    if (n > kStaticMaxN)
        return set_error(HB_EINVAL, "hash_batch_bucketed_noalloc: n exceeds the static workspace's 2^20 messages");
    if (!messages || !offsets || !lengths || !digests_out)
        return set_error(HB_EINVAL, "hash_batch_bucketed_noalloc: null device pointer");
    if (reinterpret_cast<uintptr_t>(digests_out) & 3u)
        return set_error(HB_EINVAL, "hash_batch_bucketed_noalloc: digests_out must be 4-byte aligned");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hash_batch_bucketed_noalloc: hipGetDevice");
    StaticDevice *sd = static_device(dev);
    if (!sd) return set_error(HB_EINVAL, "hash_batch_bucketed_noalloc: device index out of range");
    if (sd->status != HB_OK) return set_error(sd->status, sd->why);
    // a plan object on the stack: launch settings only, its workspace is the static array
    hb_plan p;
    p.ws = static_ws(sd->ptr, sd->cus);
    p.flags = HB_PLAN_LONG_INLINE;
    p.device = dev;
    p.cus = sd->cus;
    p.long_on = true;
    p.long_sched = false;
    p.long_min_key = 256;
    p.side = nullptr;  // long chains and bulk in one launch
    PlanDesc d{};
    d.algos = algos;
    d.msgs = messages;
    d.offs = offsets;
    d.lens = lengths;
    d.out = digests_out;
    d.n = n;
    d.stride = algos ? 32u : uint32_t(digest_size(algo));
    d.algo = algos ? 0 : algo;
    d.sort = 1;
    d.mpl = p.mpl;
    d.long_min_key = p.long_min_key;
    d.bulk_margin = p.bulk_margin;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_set_desc, dim3(1), dim3(1), 0, s, d, p.ws.desc);
    e = hipGetLastError();
    if (e == hipSuccess) e = enqueue_pipeline(&p, s, false);
    if (e != hipSuccess) return hip_error(e, "hash_batch_bucketed_noalloc: launch");
    return HB_OK;
}

}  // extern "C"
