// Host-only checks of the serving loop's decisions (admission in arrival order under a
// budget and a slot limit; step launches per request class) against a simulated clock and
// simulated device streams: every decision keeps the stated rules, and every request of a
// random open-loop workload completes.
#include <cassert>
#include <cstdio>
#include <deque>
#include <random>
#include <vector>

#include "../../paper_2407_09333_amd/csrc/hb_policy.hpp"

namespace {

struct Req {
    uint64_t id = 0, payload = 0, arena_off = 0;
    int cls = 0;
    double arrive = 0, staged_at = -1, done_at = -1;
};

struct Stream {
    bool busy = false;
    double until = 0;
    std::vector<Req *> step;
};

void check_decision(const hb::LaunchInputs &in, const int *launch)
{
    bool any_busy = false;
    for (int k = 0; k < in.n_streams; ++k) any_busy |= in.busy[k];
    auto ready = [&](int c) {
        return in.staged[c] > 0 &&
               (!any_busy || in.staged[c] >= in.min_batch || in.now - in.oldest_staged[c] >= in.max_wait);
    };
    auto idle_of = [&](int c) {
        for (int k = 0; k < in.n_streams; ++k)
            if (hb::stream_class(k) == c && !in.busy[k]) return true;
        return false;
    };
    int launches[2] = {0, 0};
    for (int k = 0; k < in.n_streams; ++k) {
        const int c = launch[k];
        if (c < 0) continue;
        assert(c == 0 || c == 1);
        assert(!in.busy[k]);               // never on a busy stream
        assert(ready(c));                  // only a ready class launches
        ++launches[c];
        if (c != hb::stream_class(k)) {    // taking the other class's step
            assert(in.staged[hb::stream_class(k)] == 0);
            assert(!idle_of(c));
        }
    }
    for (int c = 0; c < 2; ++c) {
        assert(launches[c] <= 1);          // one step per class per decision
        if (ready(c) && idle_of(c)) assert(launches[c] == 1);  // a ready class with an idle stream launches
    }
}

}  // namespace

int main()
{
    // fixed cases
    {
        bool busy[2] = {false, false};
        hb::LaunchInputs in;
        in.n_streams = 2;
        in.busy = busy;
        in.staged[1] = 1;
        in.oldest_staged[1] = 0.0;
        in.now = 1e-6;
        int launch[2];
        hb::choose_launches(in, launch);  // nothing running: a single staged request goes at once
        assert(launch[0] == -1 && launch[1] == 1);
        busy[1] = true;
        in.staged[1] = 3;
        hb::choose_launches(in, launch);  // long stream busy, 3 < 8 staged, not waited enough
        assert(launch[0] == -1 && launch[1] == -1);
        in.now = 1e-3;
        hb::choose_launches(in, launch);  // waited 1 ms: the idle short stream takes it
        assert(launch[0] == 1 && launch[1] == -1);
        in.staged[0] = 1;
        in.oldest_staged[0] = in.now;
        hb::choose_launches(in, launch);  // its own class has one (not ready): it waits for it
        assert(launch[0] == -1);
    }
    // admission: in order, within budget and slots, stops at the first misfit
    {
        hb::Arena arena(10000);
        std::deque<Req *> pending;
        std::vector<Req> rs(6);
        const uint64_t pay[6] = {3000, 2000, 0, 6000, 100, 100};
        for (int i = 0; i < 6; ++i) {
            rs[i].id = uint64_t(i);
            rs[i].payload = pay[i];
            pending.push_back(&rs[i]);
        }
        int slots = 0;
        std::vector<uint64_t> order;
        size_t n = hb::admit_in_order(pending, arena, slots, 8, [&](Req *r) { order.push_back(r->id); });
        // 3072 + 2048 + (none) = 5120 used; 6144 does not fit: 4 and 5 wait behind it
        assert(n == 3 && slots == 3 && order == (std::vector<uint64_t>{0, 1, 2}));
        assert(pending.front()->id == 3);
        arena.release(rs[0].arena_off, rs[0].payload);  // 0 and 1 finish
        arena.release(rs[1].arena_off, rs[1].payload);
        slots -= 2;
        n = hb::admit_in_order(pending, arena, slots, 3, [&](Req *r) { order.push_back(r->id); });
        assert(n == 2 && slots == 3 && pending.front()->id == 5);  // the slot limit stops 5
        assert(order == (std::vector<uint64_t>{0, 1, 2, 3, 4}));
    }
    // simulation: random open-loop arrivals, staging delays and step durations
    std::mt19937_64 rng(17);
    long decisions = 0, completed = 0;
    for (int run = 0; run < 40; ++run) {
        const int n_streams = 2 + int(rng() % 3);
        const uint64_t budget = 1 << (20 + rng() % 4);
        const int max_slots = 4 + int(rng() % 60);
        hb::Arena arena(budget);
        std::vector<Req> reqs(2000);
        double t = 0;
        for (size_t i = 0; i < reqs.size(); ++i) {
            t += std::exponential_distribution<double>(20000.0)(rng);
            reqs[i].id = i;
            reqs[i].arrive = t;
            reqs[i].payload = (rng() % 8 == 0) ? 0 : 1 + rng() % (budget / 4);
            reqs[i].cls = int(rng() % 3 == 0);
        }
        std::deque<Req *> pending, staging;
        std::vector<Req *> staged[2];
        std::vector<Stream> st(static_cast<size_t>(n_streams));
        int slots = 0;
        size_t next = 0;
        uint64_t last_admitted = 0;
        bool any_admitted = false;
        double now = 0;
        const double dt = 20e-6;
        while (completed < long(reqs.size()) * (run + 1)) {
            now += dt;
            while (next < reqs.size() && reqs[next].arrive <= now) pending.push_back(&reqs[next++]);
            // completions
            for (Stream &s : st) {
                if (!s.busy || s.until > now) continue;
                for (Req *r : s.step) {
                    r->done_at = now;
                    if (r->payload) arena.release(r->arena_off, r->payload);
                    --slots;
                    ++completed;
                }
                s.step.clear();
                s.busy = false;
            }
            // admission
            hb::admit_in_order(pending, arena, slots, max_slots, [&](Req *r) {
                assert(!any_admitted || r->id == last_admitted + 1);  // arrival order
                last_admitted = r->id;
                any_admitted = true;
                staging.push_back(r);
            });
            assert(arena.used() <= arena.capacity() && slots <= max_slots);
            if (!pending.empty() && slots < max_slots)  // held back only by the budget
                assert(arena.largest_free() < hb::Arena::round_up(pending.front()->payload));
            // staging takes a random 0-100 us per request, in order
            while (!staging.empty() && (rng() % 4 != 0)) {
                Req *r = staging.front();
                staging.pop_front();
                r->staged_at = now;
                staged[r->cls].push_back(r);
            }
            // launch decision
            bool busy[8];
            for (int k = 0; k < n_streams; ++k) busy[k] = st[size_t(k)].busy;
            hb::LaunchInputs in;
            in.n_streams = n_streams;
            in.busy = busy;
            for (int c = 0; c < 2; ++c) {
                in.staged[c] = staged[c].size();
                in.oldest_staged[c] = staged[c].empty() ? 0 : staged[c].front()->staged_at;
            }
            in.now = now;
            int launch[8];
            hb::choose_launches(in, launch);
            check_decision(in, launch);
            ++decisions;
            for (int k = 0; k < n_streams; ++k) {
                if (launch[k] < 0) continue;
                Stream &s = st[size_t(k)];
                s.step.swap(staged[launch[k]]);
                staged[launch[k]].clear();
                s.busy = true;
                s.until = now + (launch[k] ? 2e-3 : 3e-4) * (0.2 + double(rng() % 100) / 100.0);
            }
            assert(now < 1000.0);  // every request completes
        }
        for (const Req &r : reqs) assert(r.done_at >= r.arrive);
    }
    std::printf("policy ok: %ld decisions, %ld requests\n", decisions, completed);
    return 0;
}
