// hb_arena.hpp -- first-fit range allocator over a fixed device budget (host logic only).
//
// The serving loop admits a request only if its payload fits in the device arena; ranges
// are returned when the request's step completes.  Free ranges are kept sorted by offset
// and merged with their neighbours on release.  Header-only and free of HIP calls so its
// behaviour can be checked on the host.
#pragma once

#include <cstdint>
#include <iterator>
#include <map>

namespace hb {

class Arena {
public:
    static constexpr uint64_t kAlign = 256;
    static constexpr uint64_t kFail = ~uint64_t(0);

    explicit Arena(uint64_t capacity = 0) { reset(capacity); }

    void reset(uint64_t capacity)
    {
        cap_ = capacity / kAlign * kAlign;
        free_.clear();
        if (cap_) free_[0] = cap_;
        used_ = 0;
        peak_ = 0;
    }

    static uint64_t round_up(uint64_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

    // Offset of a range of at least n bytes (n == 0 takes kAlign), or kFail.
    uint64_t alloc(uint64_t n)
    {
        n = round_up(n ? n : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                const uint64_t off = it->first, rest = it->second - n;
                free_.erase(it);
                if (rest) free_[off + n] = rest;
                used_ += n;
                if (used_ > peak_) peak_ = used_;
                return off;
            }
        }
        return kFail;
    }

    // Return [off, off + n) (n as passed to alloc).
    void release(uint64_t off, uint64_t n)
    {
        n = round_up(n ? n : 1);
        used_ -= n;
        auto next = free_.lower_bound(off);
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                off = prev->first;
                n += prev->second;
                free_.erase(prev);
            }
        }
        if (next != free_.end() && off + n == next->first) {
            n += next->second;
            free_.erase(next);
        }
        free_[off] = n;
    }

    uint64_t capacity() const { return cap_; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }
    uint64_t largest_free() const
    {
        uint64_t m = 0;
        for (auto &kv : free_)
            if (kv.second > m) m = kv.second;
        return m;
    }
    size_t fragments() const { return free_.size(); }

private:
    uint64_t cap_ = 0, used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

}  // namespace hb
