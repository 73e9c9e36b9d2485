// Host-only checks of the serving loop's group packing: random groups of requests (packed
// or scattered messages, empty messages, requests without payload) get arena ranges from
// the allocator, are packed piece by piece with random piece sizes into exactly-sized
// buffers, and every message byte must land at its arena position.
#include <cassert>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "../../paper_2407_09333_amd/csrc/hb_arena.hpp"
#include "../../paper_2407_09333_amd/csrc/hb_stage.hpp"

struct R {
    const uint8_t *msgs = nullptr;
    const uint64_t *offs = nullptr, *lens = nullptr;
    uint64_t n = 0, payload = 0, arena_off = 0;
    std::vector<uint8_t> mem;
    std::vector<uint64_t> o, l;
};

int main()
{
    std::mt19937_64 rng(11);
    long groups = 0, pieces = 0;
    for (int it = 0; it < 3000; ++it) {
        const int k = 1 + int(rng() % 9);
        std::vector<R> reqs(k);
        hb::Arena arena(1 << 20);
        const uint64_t skip = rng() % 3000;  // the group need not start at offset 0
        if (skip) arena.alloc(skip);
        for (R &r : reqs) {
            const int kind = int(rng() % 5);  // 0: no messages, 1: all empty, else random
            r.n = kind == 0 ? 0 : 1 + rng() % 40;
            for (uint64_t i = 0; i < r.n; ++i) r.l.push_back(kind == 1 ? 0 : (rng() % 4 == 0 ? 0 : rng() % 700));
            const bool scattered = rng() % 2;
            uint64_t pos = 0;
            for (uint64_t i = 0; i < r.n; ++i) {
                if (scattered) pos += rng() % 17;
                r.o.push_back(pos);
                pos += r.l[i];
            }
            r.mem.resize(pos + 1);
            for (auto &b : r.mem) b = uint8_t(rng());
            r.msgs = r.mem.data();
            r.offs = r.o.data();
            r.lens = r.l.data();
            for (uint64_t x : r.l) r.payload += x;
            r.arena_off = r.payload ? arena.alloc(r.payload) : 0;
            assert(r.arena_off != hb::Arena::kFail);
        }
        std::vector<const R *> ptr;
        for (const R &r : reqs) ptr.push_back(&r);
        hb::GroupPacker<R> pk(ptr.data(), k);
        std::vector<uint8_t> dev(1 << 20, 0xEE);  // the arena as the copies leave it
        while (pk.done() < pk.total()) {
            const uint64_t cap = 1 + rng() % 2500;
            const uint64_t want = std::min<uint64_t>(cap, pk.total() - pk.done());
            std::vector<uint8_t> piece(want);  // exactly sized: a write past it trips ASan
            const uint64_t at = pk.dst0() + pk.done();
            const uint64_t got = pk.next(piece.data(), cap);
            assert(got == want);
            std::memcpy(dev.data() + at, piece.data(), got);
            ++pieces;
        }
        for (const R &r : reqs) {
            uint64_t pos = r.arena_off;
            for (uint64_t i = 0; i < r.n; ++i) {
                assert(std::memcmp(dev.data() + pos, r.msgs + r.offs[i], r.l[i]) == 0);
                pos += r.l[i];
            }
        }
        ++groups;
    }
    std::printf("stage ok: %ld groups, %ld pieces\n", groups, pieces);
    return 0;
}
