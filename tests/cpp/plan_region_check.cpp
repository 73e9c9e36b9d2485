// Host model of the batched plan's long-chain scratch assignment (k_long_scan): the
// messages of one algorithm in bucketed order (block-count keys descending, saturated keys
// in arbitrary order), taken a wave of 64 at a time while the waves' regions fit the
// scratch.  Checks, over random and hand-made orders, that every lane's block count fits
// its wave's region, that regions are disjoint and inside the scratch -- and shows that the
// earlier rule (region = lane 0's block count) breaks this once keys saturate.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2407_09333_amd/csrc/hb_plan_rules.hpp"

namespace {

struct Assignment {
    std::vector<uint64_t> base;  // per taken wave
    uint64_t end = 0;
};

// The scan of k_long_scan for one segment: region per wave by `rule`, prefix sums, and
// the fitting prefix of waves.
template <class Rule>
Assignment assign(const std::vector<uint64_t> &sorted_lens, uint32_t cand, uint64_t cap, uint64_t max_waves,
                  Rule rule)
{
    Assignment a;
    const uint32_t nw = (cand + 63u) / 64u;
    uint64_t run = 0;
    for (uint32_t w = 0; w < nw && w < max_waves; ++w) {
        const uint32_t lanes = std::min<uint32_t>(64u, cand - w * 64u);
        const uint64_t r = rule(&sorted_lens[size_t(w) * 64u], lanes, cap + 1);
        if (run + r > cap) break;
        a.base.push_back(run);
        run += r;
    }
    a.end = run;
    return a;
}

uint64_t rule_max(const uint64_t *lens, uint32_t lanes, uint64_t limit)
{
    return hb::wave_region_blocks([&](uint32_t l) { return lens[l]; }, lanes, limit);
}

uint64_t rule_first_lane(const uint64_t *lens, uint32_t, uint64_t limit)
{
    const uint64_t r = hb::block_count(lens[0]);
    return r < limit ? r : limit;
}

// Lanes whose block count exceeds their wave's region (reads past it).
uint64_t overruns(const std::vector<uint64_t> &sorted_lens, uint32_t cand, const Assignment &a)
{
    uint64_t bad = 0;
    for (size_t w = 0; w < a.base.size(); ++w) {
        const uint64_t region = (w + 1 < a.base.size() ? a.base[w + 1] : a.end) - a.base[w];
        for (uint32_t l = 0; l < 64u && w * 64u + l < cand; ++l)
            if (hb::block_count(sorted_lens[w * 64u + l]) > region) ++bad;
    }
    return bad;
}

// Bucketed order of a segment: keys descending; inside the saturated key the order is
// whatever the atomics gave, modelled by `shuffle` (or index order).
std::vector<uint64_t> bucketed(std::vector<uint64_t> lens, std::mt19937_64 *shuffle)
{
    std::stable_sort(lens.begin(), lens.end(),
                     [](uint64_t x, uint64_t y) { return hb::sort_key(x) > hb::sort_key(y); });
    if (shuffle) {
        auto sat_end = std::find_if(lens.begin(), lens.end(),
                                    [](uint64_t x) { return hb::sort_key(x) < hb::kBins - 1; });
        std::shuffle(lens.begin(), sat_end, *shuffle);
    }
    return lens;
}

int fail(const char *what)
{
    std::printf("FAIL: %s\n", what);
    return 1;
}

}  // namespace

int main()
{
    // Rule basics.
    if (hb::block_count(0) != 1 || hb::block_count(55) != 1 || hb::block_count(56) != 2 ||
        hb::block_count(119) != 2 || hb::block_count(120) != 3)
        return fail("block_count");
    const uint64_t sat_len = uint64_t(hb::kBins - 1 - 1) * 64u - 8u;  // smallest length of key kBins - 1
    if (hb::sort_key(sat_len) != hb::kBins - 1 || hb::sort_key(sat_len - 1) != hb::kBins - 2)
        return fail("sort_key saturation point");
    std::printf("saturated key from L = %llu bytes\n", (unsigned long long)sat_len);

    const uint64_t cap = 32768;  // 1 GiB of 32 KiB wave-blocks
    const uint32_t min_key = 256;

    // The defect: a 1.5 MiB message ordered ahead of a 3 MiB one in the same wave.
    {
        std::vector<uint64_t> lens{3ull << 19, 3ull << 20};
        for (int i = 0; i < 62; ++i) lens.push_back((1ull << 20) + 4096u * uint64_t(i + 1));
        std::vector<uint64_t> order = lens;  // index order inside the saturated key
        const uint64_t first = rule_first_lane(order.data(), 64, cap + 1);
        const uint64_t need = rule_max(order.data(), 64, cap * 4);
        std::printf("first-lane rule: region %llu wave-blocks, longest lane needs %llu\n",
                    (unsigned long long)first, (unsigned long long)need);
        if (first != 24577 || need != 49153) return fail("worked example sizes");
        const Assignment old_a = assign(order, 64, cap, 1u << 20, rule_first_lane);
        if (old_a.base.size() != 1 || overruns(order, 64, old_a) == 0)
            return fail("the first-lane rule should overrun on the worked example");
        const Assignment new_a = assign(order, 64, cap, 1u << 20, rule_max);
        if (!new_a.base.empty()) return fail("a 49,153-block wave must not fit a 32,768-block scratch");
        const Assignment big = assign(order, 64, 4 * cap, 1u << 20, rule_max);
        if (big.base.size() != 1 || big.end != 49153 || overruns(order, 64, big) != 0)
            return fail("max rule with a larger scratch");
        std::printf("first-lane rule overruns %llu lanes; max rule: no overrun\n",
                    (unsigned long long)overruns(order, 64, old_a));
    }

    // Random segments: mixes of saturated and unsaturated long messages, random orders
    // inside the saturated key, several scratch sizes.
    std::mt19937_64 rng(2407);
    uint64_t old_bad_cases = 0;
    for (int trial = 0; trial < 3000; ++trial) {
        const int n = 1 + int(rng() % 400);
        std::vector<uint64_t> lens(n);
        for (auto &L : lens) {
            switch (rng() % 4) {
            case 0: L = rng() % (64u * 300u); break;                       // short or around the threshold
            case 1: L = (1ull << 20) + rng() % (1ull << 20); break;        // at or past saturation
            case 2: L = (1ull << 21) + rng() % (3ull << 20); break;        // 2 - 5 MiB
            default: L = 16384u + rng() % (1ull << 20); break;             // below saturation
            }
        }
        std::vector<uint64_t> order = bucketed(lens, (trial & 1) ? &rng : nullptr);
        uint32_t cand = 0;
        for (uint64_t L : order) cand += hb::sort_key(L) >= min_key;
        const uint64_t caps[] = {1024, cap, 8 * cap, 1ull << 32};
        for (uint64_t c : caps) {
            const Assignment a = assign(order, cand, c, 1u << 20, rule_max);
            if (overruns(order, cand, a) != 0) return fail("max rule overrun");
            if (a.end > c) return fail("regions past the scratch");
            for (size_t w = 1; w < a.base.size(); ++w)
                if (a.base[w] < a.base[w - 1]) return fail("regions out of order");
            // keys are sorted descending, so an unsaturated lane 0 bounds its wave exactly
            for (size_t w = 0; w < a.base.size(); ++w)
                if (hb::sort_key(order[w * 64]) < hb::kBins - 1) {
                    const uint64_t region = (w + 1 < a.base.size() ? a.base[w + 1] : a.end) - a.base[w];
                    if (region != hb::block_count(order[w * 64])) return fail("unsaturated region");
                }
            old_bad_cases += overruns(order, cand, assign(order, cand, c, 1u << 20, rule_first_lane)) > 0;
        }
    }
    if (old_bad_cases == 0) return fail("random orders never exposed the first-lane rule");
    std::printf("random segments: max rule never overruns; first-lane rule overran in %llu cases\n",
                (unsigned long long)old_bad_cases);
    std::printf("plan region ok\n");
    return 0;
}
