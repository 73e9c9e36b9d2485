// hb_policy.hpp -- the serving loop's decisions: admission and step launches (host logic
// only, free of HIP calls so they can be checked on the host with a simulated clock).
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>

#include "hb_arena.hpp"

namespace hb {

// Admission in arrival order: the head of `pending` is admitted while a slot is free and
// its payload fits the arena; the first request that does not fit stops admission (no
// request overtakes another).  R needs `payload` and `arena_off` members; `on_admit(r)` is
// called for each admitted request after its range is reserved.  Returns the number
// admitted.
// `take_more(r)` (optional) reserves any further resource the request needs after its arena
// range; if it returns false the range is given back and admission stops there too.
struct TakeNothing {
    template <class R> bool operator()(R *) const { return true; }
};

template <class R, class F, class T = TakeNothing>
size_t admit_in_order(std::deque<R *> &pending, Arena &arena, int &slots_used, int max_slots, F &&on_admit,
                      T &&take_more = T())
{
    size_t admitted = 0;
    while (!pending.empty() && slots_used < max_slots) {
        R *r = pending.front();
        uint64_t off = 0;
        if (r->payload) {
            off = arena.alloc(r->payload);
            if (off == Arena::kFail) break;
        }
        if (!take_more(r)) {
            if (r->payload) arena.release(off, r->payload);
            break;
        }
        r->arena_off = off;
        ++slots_used;
        pending.pop_front();
        on_admit(r);
        ++admitted;
    }
    return admitted;
}

// Step launches.  Stream 0 serves short-chain steps (class 0), the others long-chain ones
// (class 1).  A class launches a step on an idle stream of its own when either no step is
// running anywhere, at least min_batch of its requests are staged, or its oldest staged
// request has waited max_wait; at most one step per class per decision.  An idle stream
// whose class has nothing staged takes a ready step of the other class while all of that
// class's streams are busy.
struct LaunchInputs {
    int n_streams = 0;
    const bool *busy = nullptr;          // per stream
    size_t staged[2] = {0, 0};           // staged requests per class
    double oldest_staged[2] = {0, 0};    // staging time of each class's oldest
    double now = 0;
    size_t min_batch = 8;
    double max_wait = 200e-6;
};

inline int stream_class(int k) { return k == 0 ? 0 : 1; }

// Fills launch_cls[0, n_streams) with the class to launch on each stream (-1: none).
inline void choose_launches(const LaunchInputs &in, int *launch_cls)
{
    bool any_busy = false;
    for (int k = 0; k < in.n_streams; ++k) {
        launch_cls[k] = -1;
        any_busy |= in.busy[k];
    }
    auto ready = [&](int c) {
        return in.staged[c] > 0 &&
               (!any_busy || in.staged[c] >= in.min_batch || in.now - in.oldest_staged[c] >= in.max_wait);
    };
    auto all_busy = [&](int c) {
        for (int k = 0; k < in.n_streams; ++k)
            if (stream_class(k) == c && !in.busy[k]) return false;
        return true;
    };
    bool launched[2] = {false, false};
    for (int k = 0; k < in.n_streams; ++k) {
        if (in.busy[k]) continue;
        const int c = stream_class(k), o = 1 - c;
        if (!launched[c] && ready(c)) {
            launch_cls[k] = c;
            launched[c] = true;
        } else if (in.staged[c] == 0 && !launched[o] && all_busy(o) && ready(o)) {
            launch_cls[k] = o;
            launched[o] = true;
        }
    }
}

}  // namespace hb
