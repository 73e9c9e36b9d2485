// hb_stage.hpp -- packing a group of serving requests into staging memory laid out like
// their arena ranges (host logic only, free of HIP calls so it can be checked on the host).
//
// A group is a run of admitted requests whose arena ranges follow each other: each starts
// where the previous one's range, rounded up to the allocator's alignment, ends.  Requests
// without payload may sit anywhere in the run and take no space.  Request q's messages
// lie back to back from its arena offset, in index order, so the group is one byte range
// [dst0, dst0 + total) of the arena; the packer fills it piece by piece, leaving the
// alignment gaps between requests unwritten (nothing reads them).
#pragma once

#include <algorithm>
#include <cstdint>
#include <cstring>

namespace hb {

// R: any type with msgs (const uint8_t *), offs / lens (const uint64_t *), n, payload and
// arena_off (uint64_t) members.
template <class R>
class GroupPacker {
public:
    GroupPacker(const R *const *rs, int k) : rs_(rs), k_(k)
    {
        bool have = false;
        for (int q = 0; q < k; ++q) {
            if (!rs[q]->payload) continue;
            if (!have) { dst0_ = rs[q]->arena_off; have = true; }
            total_ = rs[q]->arena_off + rs[q]->payload - dst0_;
        }
    }

    uint64_t dst0() const { return dst0_; }    // arena offset of the group's first byte
    uint64_t total() const { return total_; }  // bytes from dst0 to the last payload byte
    uint64_t done() const { return done_; }    // bytes handed out so far

    // Fill buf[0, m) with the group's next m = min(cap, total - done) bytes; returns m
    // (fewer only if the requests do not hold what their arena ranges promise).
    // Message bytes come from one memcpy per run of messages that are contiguous in the
    // caller's memory (a packed request is one run).
    uint64_t next(uint8_t *buf, uint64_t cap)
    {
        const uint64_t want = std::min<uint64_t>(cap, total_ - done_);
        uint64_t filled = 0;
        while (filled < want && ri_ < k_) {
            const R *r = rs_[ri_];
            if (i_ >= r->n || !r->payload) {
                ++ri_;
                i_ = within_ = rbytes_ = 0;
                continue;
            }
            // alignment gap before this request's range
            const uint64_t target = r->arena_off - dst0_ + rbytes_;
            if (done_ + filled < target) {
                filled += std::min<uint64_t>(target - (done_ + filled), want - filled);
                continue;
            }
            const uint8_t *src = r->msgs + r->offs[i_] + within_;
            uint64_t run = 0;
            while (filled + run < want && i_ < r->n && r->msgs + r->offs[i_] + within_ == src + run) {
                const uint64_t take = std::min<uint64_t>(r->lens[i_] - within_, want - filled - run);
                run += take;
                within_ += take;
                if (within_ == r->lens[i_]) { ++i_; within_ = 0; }
                else break;
            }
            if (run) std::memcpy(buf + filled, src, run);
            filled += run;
            rbytes_ += run;
        }
        done_ += filled;
        return filled;
    }

private:
    const R *const *rs_;
    int k_;
    uint64_t dst0_ = 0, total_ = 0, done_ = 0;
    int ri_ = 0;                                    // request of the cursor
    uint64_t i_ = 0, within_ = 0, rbytes_ = 0;      // message in it, bytes of that message
                                                    // and of the request already packed
};

}  // namespace hb
