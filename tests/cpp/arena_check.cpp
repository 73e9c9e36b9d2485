// Host-only checks of the serving arena (first-fit allocator with coalescing).
#include <cassert>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_2407_09333_amd/csrc/hb_arena.hpp"

int main()
{
    using hb::Arena;
    Arena a(1 << 20);
    assert(a.capacity() == (1 << 20));
    uint64_t x = a.alloc(1000), y = a.alloc(5000), z = a.alloc(1);
    assert(x == 0 && y == 1024 && z == 1024 + 5120);
    assert(a.used() == 1024 + 5120 + 256);
    a.release(y, 5000);
    assert(a.alloc(6000) == 1024 + 5120 + 256);  // hole too small: goes after z
    assert(a.alloc(5000) == 1024);               // first fit reuses the hole
    // over budget fails, nothing changes
    uint64_t used = a.used();
    assert(a.alloc(1 << 20) == Arena::kFail && a.used() == used);
    // random alloc/free never overlaps and coalesces back to one range
    std::mt19937_64 rng(5);
    Arena b(64 << 20);
    std::vector<std::pair<uint64_t, uint64_t>> live;
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || (rng() % 3)) {
            uint64_t n = 1 + rng() % (1 << 20);
            uint64_t off = b.alloc(n);
            if (off == Arena::kFail) continue;
            for (auto &p : live) assert(off + Arena::round_up(n) <= p.first || p.first + Arena::round_up(p.second) <= off);
            assert(off + n <= b.capacity());
            live.push_back({off, n});
        } else {
            size_t k = rng() % live.size();
            b.release(live[k].first, live[k].second);
            live.erase(live.begin() + k);
        }
        assert(b.used() <= b.capacity() && b.peak() >= b.used());
    }
    for (auto &p : live) b.release(p.first, p.second);
    assert(b.used() == 0 && b.fragments() == 1 && b.largest_free() == b.capacity());
    std::printf("arena ok\n");
    return 0;
}
