// hb_serve.hpp -- layout shared by the serving loop (host) and the resident serving kernel
// (device): the work-item ring the host publishes into and the per-message rings the items
// point at.  Free of HIP calls.
#pragma once

#include <stdint.h>

namespace hb {

// An item whose longest message has at least kServeCoopBlocks blocks and which holds at
// most kServeCoopMaxMessages messages is hashed by the whole wave together (the schedule
// words of a window of blocks computed by all lanes, the chains running rounds only):
// a shorter critical path per chain, at the cost of lanes left idle.  Each window then
// holds >= 16 blocks per chain, so its load latency is amortised.
constexpr int kServeThreads = 256;  // threads per workgroup of the serving kernel (four waves)
constexpr uint64_t kServeCoopBlocks = 128;
constexpr uint32_t kServeCoopMaxMessages = 4;

// One work item: up to 64 messages of one algorithm, one per lane, taken from message
// slots first .. first + count - 1 of the rings below.
struct ServeItem {
    uint32_t first;   // first message slot
    uint32_t count;   // 1 .. 64
    uint32_t algo;    // 0 MD5, 1 SHA-1, 2 SM3
    uint32_t blocks;  // block count of its longest message (capped at 2^32 - 1): how long
                      // the item runs, which decides its path and how a wave claims it
};

// A wave that finds a backlog claims several consecutive items at once, but only while
// their summed `blocks` stay within this budget: items come longest first, and long items
// claimed together would run one after another on one wave while others idle.
constexpr uint32_t kServeClaimBlocks = 64;

// Everything the resident kernel reads or writes, as device addresses.  "Host" rings are
// pinned, coherent host memory reached through its device mapping; the host writes items
// and message slots there and reads digests and done flags back without any copy.
struct ServeRings {
    const ServeItem *h_items;   // item ring written by the host (items_cap entries)
    const uint64_t *h_tail;     // items published so far (host-written, monotone)
    const uint32_t *h_stop;     // nonzero: the host asks the kernel to exit
    uint32_t *done;             // per item ring entry: its ring position + 1 once hashed
    const uint64_t *off;        // per message slot: byte offset of the message in the arena
    const uint64_t *len;        // per message slot: its length
    uint8_t *digests;           // digest ring, 32 bytes per message slot (bytes past the digest
                                // zeroed), in slot order: the host maps slots back to the
                                // caller's message order
    const uint8_t *arena;       // device arena holding the payload
    ServeItem *d_items;         // device copy of the item ring
    uint64_t *d_head;           // next item to claim (device memory, kept across launches)
    uint64_t *d_tail;           // items copied into d_items (device memory, kept across launches)
    uint32_t *d_stop;           // launch generation told to stop (device memory)
    uint64_t items_cap;         // item ring entries (a power of two)
    uint64_t idle_ticks;        // exit after this many 100 MHz ticks without a new item
    uint64_t max_ticks;         // and after this many in any case (the host relaunches)
};

}  // namespace hb
