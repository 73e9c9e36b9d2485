// hb_items.hpp -- how the resident serving mode lays out one request's messages in
// message slots and cuts them into work items (host logic only, free of HIP calls so it
// can be checked on the host).
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

#include "hb_serve.hpp"

namespace hb {

// Blocks of a message of len bytes: MD5, SHA-1 and SM3 all pad to 64-byte blocks with an
// 8-byte length field (RFC 1321 Sec. 3.1-3.2; FIPS 180-4 Sec. 5.1.1; GB/T 32905 Sec. 5.2).
inline uint64_t serve_block_count(uint64_t len) { return (len + 8) / 64 + 1; }

constexpr int kServeClasses = 64;  // power-of-two block-count classes

// Class index of a block count, longest first: class c holds block counts in
// [2^(63 - c), 2^(64 - c)).
inline int serve_class(uint64_t nb)
{
    int c = 0;
    while (nb > 1) { nb >>= 1; ++c; }
    return kServeClasses - 1 - c;
}

// One request of n messages (lens[i] bytes, algorithm algo_of(i) in 0..2).
//
// Slots: its messages take the relative slots 0 .. n - 1 ordered by algorithm and, within
// one, by block-count class, longest first (index order within a class), so the lanes of
// an item finish close together; slot_of[i] is message i's slot.
//
// Items: each algorithm's slots in runs of at most 64 messages (one per lane), each with
// its longest message's block count.  A request is done when its longest chain is, and a
// chain's blocks are sequential, so with `latency` set (the device has idle waves) each
// algorithm's messages in its two longest classes, where those have >= kServeCoopBlocks
// blocks, go first into items of at most kServeCoopMaxMessages messages, sizes differing
// by at most one: the kernel hashes such items with the whole wave on each chain's critical
// path.  Item `first` fields are relative slots (the caller adds its first slot).
template <class AlgoOf>
void form_serve_items(uint64_t n, const uint64_t *lens, AlgoOf &&algo_of, bool latency, std::vector<uint32_t> &slot_of,
                      std::vector<ServeItem> &items)
{
    std::vector<uint32_t> count(3 * kServeClasses, 0);
    for (uint64_t i = 0; i < n; ++i) count[algo_of(i) * kServeClasses + serve_class(serve_block_count(lens[i]))]++;
    std::vector<uint32_t> start(3 * kServeClasses + 1, 0);
    for (int k = 0; k < 3 * kServeClasses; ++k) start[k + 1] = start[k] + count[k];
    std::vector<uint32_t> next(start.begin(), start.end() - 1);
    std::vector<uint64_t> nb_at(n);  // block count by slot
    slot_of.resize(n);
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t nb = serve_block_count(lens[i]);
        const uint32_t k = next[algo_of(i) * kServeClasses + serve_class(nb)]++;
        slot_of[i] = k;
        nb_at[k] = nb;
    }
    items.clear();
    auto item = [&](uint32_t f, uint32_t cnt, int a) {
        uint64_t nb = 0;
        for (uint32_t k = f; k < f + cnt; ++k) nb = std::max(nb, nb_at[k]);
        items.push_back(ServeItem{f, cnt, uint32_t(a), uint32_t(std::min<uint64_t>(nb, UINT32_MAX))});
    };
    for (int a = 0; a < 3; ++a) {
        const uint32_t b = start[a * kServeClasses], e = start[(a + 1) * kServeClasses];
        uint32_t f = b;
        if (latency) {
            int c0 = 0;
            while (c0 < kServeClasses && count[a * kServeClasses + c0] == 0) ++c0;
            uint32_t top = b;  // end of the messages taken cooperatively
            for (int c = c0; c < c0 + 2 && c < kServeClasses; ++c)
                if ((uint64_t(1) << (kServeClasses - 1 - c)) >= kServeCoopBlocks) top = start[a * kServeClasses + c + 1];
            const uint32_t n_top = top - b;
            if (n_top > 0) {
                const uint32_t k = (n_top + kServeCoopMaxMessages - 1) / kServeCoopMaxMessages;  // items
                for (uint32_t q = 0; q < k; ++q) {
                    const uint32_t lo = b + uint32_t(uint64_t(n_top) * q / k), hi = b + uint32_t(uint64_t(n_top) * (q + 1) / k);
                    item(lo, hi - lo, a);
                }
                f = top;
            }
        }
        for (; f < e; f += 64) item(f, std::min<uint32_t>(64, e - f), a);
    }
}

}  // namespace hb
