// Host-only checks of the resident serving mode's slot layout and work items
// (form_serve_items) over random requests: the slots are a permutation grouped by algorithm
// and, within one, by block-count class longest first; the items cover every slot once, in
// order, each with one algorithm, at most 64 messages and its longest message's block
// count; without the latency formation every item of an algorithm but its last holds 64
// messages; with it, exactly the messages of the algorithm's two longest classes with at
// least kServeCoopBlocks blocks come first, in items of at most kServeCoopMaxMessages
// whose sizes differ by at most one.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2407_09333_amd/csrc/hb_items.hpp"

namespace {

int failures = 0;

#define CHECK(cond, ...)                                          \
    do {                                                          \
        if (!(cond)) {                                            \
            if (failures++ < 10) {                                \
                std::printf("FAIL line %d: %s: ", __LINE__, #cond); \
                std::printf(__VA_ARGS__);                         \
                std::printf("\n");                                \
            }                                                     \
        }                                                         \
    } while (0)

// the class of a block count written out as a loop over powers of two (not serve_class)
int class_of(uint64_t nb)
{
    int c = 63;
    for (uint64_t p = 2; p <= nb && p != 0; p <<= 1) --c;
    return c;
}

void check_request(const std::vector<uint64_t> &lens, const std::vector<int> &algo, bool latency)
{
    const uint64_t n = lens.size();
    std::vector<uint32_t> slot_of;
    std::vector<hb::ServeItem> items;
    hb::form_serve_items(n, lens.data(), [&](uint64_t i) { return algo[i]; }, latency, slot_of, items);
    CHECK(slot_of.size() == n, "slot_of size %zu", slot_of.size());
    std::vector<int64_t> at(n, -1);  // message index at each slot
    for (uint64_t i = 0; i < n; ++i) {
        CHECK(slot_of[i] < n, "slot %u", slot_of[i]);
        if (slot_of[i] >= n) return;
        CHECK(at[slot_of[i]] < 0, "slot %u taken twice", slot_of[i]);
        at[slot_of[i]] = int64_t(i);
    }
    auto nb = [&](uint64_t k) { return uint64_t((lens[at[k]] + 8) / 64 + 1); };
    for (uint64_t k = 1; k < n; ++k) {  // grouped by algorithm, longest class first, index order within
        const int a0 = algo[at[k - 1]], a1 = algo[at[k]];
        CHECK(a0 <= a1, "algorithms out of order at slot %llu", (unsigned long long)k);
        if (a0 == a1) {
            const int c0 = class_of(nb(k - 1)), c1 = class_of(nb(k));
            CHECK(c0 <= c1, "classes out of order at slot %llu", (unsigned long long)k);
            if (c0 == c1) CHECK(at[k - 1] < at[k], "index order within a class at slot %llu", (unsigned long long)k);
        }
    }
    // items: consecutive, covering, one algorithm each, blocks = the longest
    uint64_t next = 0;
    for (const hb::ServeItem &it : items) {
        CHECK(it.first == next, "item starts at %u, expected %llu", it.first, (unsigned long long)next);
        CHECK(it.count >= 1 && it.count <= 64, "count %u", it.count);
        uint64_t longest = 0;
        for (uint64_t k = it.first; k < uint64_t(it.first) + it.count && k < n; ++k) {
            CHECK(algo[at[k]] == int(it.algo), "algorithm mismatch in item at %u", it.first);
            longest = std::max(longest, nb(k));
        }
        CHECK(it.blocks == longest, "blocks %u, longest %llu", it.blocks, (unsigned long long)longest);
        next = uint64_t(it.first) + it.count;
    }
    CHECK(next == n, "items cover %llu of %llu", (unsigned long long)next, (unsigned long long)n);
    // per algorithm: the formation
    for (int a = 0; a < 3; ++a) {
        std::vector<const hb::ServeItem *> its;
        for (const hb::ServeItem &it : items)
            if (int(it.algo) == a) its.push_back(&it);
        if (its.empty()) continue;
        // the messages the latency formation takes cooperatively
        uint64_t b = its.front()->first, e = uint64_t(its.back()->first) + its.back()->count, top = b;
        if (latency) {
            const int c0 = class_of(nb(b));
            for (uint64_t k = b; k < e; ++k) {
                const int c = class_of(nb(k));
                if (c <= c0 + 1 && (uint64_t(1) << (63 - c)) >= hb::kServeCoopBlocks) top = k + 1;
            }
        }
        size_t q = 0;
        uint32_t lo = 64, hi = 0;
        for (; q < its.size() && its[q]->first < top; ++q) {
            CHECK(its[q]->count <= hb::kServeCoopMaxMessages, "cooperative item of %u", its[q]->count);
            CHECK(uint64_t(its[q]->first) + its[q]->count <= top, "cooperative item crosses the top classes");
            lo = std::min(lo, its[q]->count);
            hi = std::max(hi, its[q]->count);
        }
        if (q) CHECK(hi - lo <= 1, "cooperative item sizes %u..%u", lo, hi);
        if (q) CHECK(q == (top - b + hb::kServeCoopMaxMessages - 1) / hb::kServeCoopMaxMessages, "%zu cooperative items", q);
        for (size_t r = q; r < its.size(); ++r)
            CHECK(its[r]->count == 64 || r + 1 == its.size(), "item of %u before the algorithm's last", its[r]->count);
    }
}

}  // namespace

int main()
{
    std::mt19937_64 rng(11);
    std::normal_distribution<double> z(0.0, 1.5);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    int requests = 0;
    for (int t = 0; t < 3000; ++t) {
        const uint64_t n = t < 10 ? uint64_t(t) : 1 + uint64_t(std::exp(u(rng) * std::log(12000.0)));
        const int single = int(rng() % 4) - 1;  // -1: mixed algorithms
        std::vector<uint64_t> lens(n);
        std::vector<int> algo(n);
        const double median = (t % 3 == 0) ? 256.0 : (t % 3 == 1 ? 8192.0 : 40000.0);
        for (uint64_t i = 0; i < n; ++i) {
            uint64_t L = uint64_t(std::exp(std::log(median) + z(rng)));
            if (rng() % 40 == 0) L = 0;
            lens[i] = std::min<uint64_t>(L, t % 7 == 0 ? (uint64_t(1) << 24) : 65536);
            algo[i] = single >= 0 ? single : int(rng() % 3);
        }
        check_request(lens, algo, false);
        check_request(lens, algo, true);
        ++requests;
    }
    // a class boundary case: the two longest classes just at and below kServeCoopBlocks
    {
        std::vector<uint64_t> lens;
        for (int i = 0; i < 9; ++i) lens.push_back((hb::kServeCoopBlocks - 1) * 64 - 8);   // 128 blocks
        for (int i = 0; i < 5; ++i) lens.push_back((hb::kServeCoopBlocks - 1) * 64 - 72);  // 127 blocks
        for (int i = 0; i < 70; ++i) lens.push_back(100);
        std::vector<int> algo(lens.size(), 2);
        check_request(lens, algo, true);
        std::vector<uint32_t> slot_of;
        std::vector<hb::ServeItem> items;
        hb::form_serve_items(lens.size(), lens.data(), [&](uint64_t i) { return algo[i]; }, true, slot_of, items);
        CHECK(items.size() >= 3 && items[0].count == 3 && items[1].count == 3 && items[2].count == 3,
              "nine 128-block messages in three items of three");
        CHECK(items.size() >= 4 && items[3].blocks == 127 && items[3].count == 64, "the 127-block class starts the full items");
    }
    if (failures) {
        std::printf("items check FAILED (%d)\n", failures);
        return 1;
    }
    std::printf("items ok: %d requests, both formations\n", requests);
    return 0;
}
