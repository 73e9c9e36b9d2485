// The serving loop (hb_server.cpp, compiled unchanged) on the CPU, against a host-only
// stand-in for the HIP runtime (fakehip/) and for the library's hashing: streams are
// in-order op queues on host threads, copies are memcpy, a plan run writes a keyed
// checksum of each message in place of its digest.  Checks, under random open-loop
// traffic from several client threads with admission stalls and cancels:
//  - every request's "digests" are its own messages' checksums, slot by slot (the arena,
//    the staging rings, the step metadata and the digest copy-back route bytes right);
//  - the event and stream rules: no event destroyed while its record or a wait on it is
//    outstanding, no event recorded again while its last record is in flight, no wait on
//    an event never recorded, no use of a destroyed stream or event.
// Run under ThreadSanitizer or AddressSanitizer + UBSan by the Python test.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "../../include/hb.h"
#include "fakehip/fake_hip.hpp"
#include "../../paper_2407_09333_amd/csrc/hb_serve.hpp"

// ---- stand-ins for the rest of libhb that the serving loop calls -------------------------

namespace hb {
static thread_local std::string t_err;
int set_error(int status, const std::string &msg)
{
    t_err = msg;
    return status;
}
int hip_error(hipError_t e, const char *what)
{
    t_err = std::string(what) + ": " + hipGetErrorString(e);
    return HB_EHIP;
}
int digest_size(int algo) { return algo == HB_MD5 ? 16 : algo == HB_SHA1 ? 20 : algo == HB_SM3 ? 32 : 0; }
hipError_t launch_copy(void *dst, const void *src, uint64_t bytes, hipStream_t stream)
{
    return fake_hip_launch(stream, [=] { std::memcpy(dst, src, bytes); });
}
}  // namespace hb

extern "C" const char *hb_last_error(void) { return hb::t_err.c_str(); }

static void fingerprint(int algo, const uint8_t *m, uint64_t len, uint8_t *out, uint32_t stride);

// The resident serving kernel, emulated on the stand-in stream's host thread: copy newly
// published items from the host ring to the "device" ring, take them in order, write each
// message's fingerprint to its digest slot and the item's done flag, and leave when the
// host says stop or 5 ms pass without an item -- the kernel's protocol, one worker.
namespace hb {
hipError_t launch_serve(const ServeRings &R, uint32_t gen, int, hipStream_t stream)
{
    return fake_hip_launch(stream, [R, gen] {
        using clk = std::chrono::steady_clock;
        const uint64_t mask = R.items_cap - 1;
        auto last = clk::now();
        uint64_t dt = __atomic_load_n(R.d_tail, __ATOMIC_ACQUIRE);
        for (;;) {
            const uint32_t stop = __atomic_load_n(R.h_stop, __ATOMIC_ACQUIRE);
            const uint64_t ht = __atomic_load_n(R.h_tail, __ATOMIC_ACQUIRE);
            if (ht > dt) {
                for (uint64_t k = dt; k < ht; ++k) R.d_items[k & mask] = R.h_items[k & mask];
                __atomic_store_n(R.d_tail, ht, __ATOMIC_RELEASE);
                dt = ht;
            }
            uint64_t h = __atomic_load_n(R.d_head, __ATOMIC_ACQUIRE);
            for (; h < dt; ++h) {
                const ServeItem it = R.d_items[h & mask];
                for (uint32_t l = 0; l < it.count; ++l) {
                    const uint32_t slot = it.first + l;
                    fingerprint(int(it.algo), R.arena + R.off[slot], R.len[slot], R.digests + uint64_t(slot) * 32, 32);
                }
                __atomic_store_n(R.done + (h & mask), uint32_t(h + 1), __ATOMIC_RELEASE);
                __atomic_store_n(R.d_head, h + 1, __ATOMIC_RELEASE);
                last = clk::now();
            }
            if (stop || clk::now() - last > std::chrono::milliseconds(5)) break;
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
        __atomic_store_n(R.d_stop, gen, __ATOMIC_RELEASE);
    });
}
}  // namespace hb

// Keyed 64-bit FNV-1a of the message, spread over the digest size: not a hash function of
// the standards, only a per-message fingerprint that tells slots apart.
static void fingerprint(int algo, const uint8_t *m, uint64_t len, uint8_t *out, uint32_t stride)
{
    uint64_t h = 0xcbf29ce484222325ull ^ (uint64_t(algo) << 56) ^ len;
    for (uint64_t i = 0; i < len; ++i) h = (h ^ m[i]) * 0x100000001b3ull;
    const int ds = hb::digest_size(algo);
    for (int k = 0; k < ds; k += 8) {
        uint64_t z = h + uint64_t(k + 1) * 0x9e3779b97f4a7c15ull;
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z ^= z >> 31;
        std::memcpy(out + k, &z, size_t(std::min(8, ds - k)));
    }
    std::memset(out + ds, 0, stride - uint32_t(ds));
}

struct hb_plan {
    int flags;
};

extern "C" {
int hb_plan_create(hb_plan **plan, uint64_t, int flags)
{
    *plan = new hb_plan{flags};
    return HB_OK;
}
int hb_plan_run(hb_plan *, const uint8_t *algos, int algo, const uint8_t *messages, const uint64_t *offsets,
                const uint64_t *lengths, uint64_t n, uint8_t *digests_out, void *stream)
{
    const hipError_t e = fake_hip_launch(static_cast<hipStream_t>(stream), [=] {
        const uint32_t stride = algos ? 32u : uint32_t(hb::digest_size(algo));
        // a step takes time in proportion to its bytes (about 1 GB/s), so arrivals outrun
        // it and the arena budget holds requests back
        uint64_t bytes = 0;
        for (uint64_t i = 0; i < n; ++i) bytes += lengths[i];
        std::this_thread::sleep_for(std::chrono::nanoseconds(bytes));
        for (uint64_t i = 0; i < n; ++i)
            fingerprint(algos ? algos[i] : algo, messages + offsets[i], lengths[i], digests_out + i * stride, stride);
    });
    return e == hipSuccess ? HB_OK : hb::hip_error(e, "hb_plan_run");
}
void hb_plan_destroy(hb_plan *plan) { delete plan; }
}

// ---- the check ---------------------------------------------------------------------------

struct Request {
    int algo = 0;  // -1: per-message ids
    std::vector<uint8_t> algos, msgs, out;
    std::vector<uint64_t> offs, lens;
    uint64_t ticket = 0;
    bool cancelled = false;
};

static Request make_request(std::mt19937_64 &rng)
{
    Request r;
    std::uniform_real_distribution<double> u(0.0, 1.0);
    std::normal_distribution<double> z(0.0, 1.5);
    const uint64_t n = std::max<uint64_t>(1, uint64_t(std::exp(u(rng) * std::log(1500.0))));
    r.algo = int(rng() % 4) - 1;
    r.lens.resize(n);
    r.offs.resize(n);
    uint64_t total = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t L = uint64_t(std::exp(std::log(256.0) + z(rng)));
        if (rng() % 50 == 0) L = 0;
        r.lens[i] = std::min<uint64_t>(L, 16384);
        r.offs[i] = total;
        total += r.lens[i];
    }
    r.msgs.resize(std::max<uint64_t>(total, 1));
    for (auto &b : r.msgs) b = uint8_t(rng());
    if (r.algo < 0) {
        r.algos.resize(n);
        for (auto &a : r.algos) a = uint8_t(rng() % 3);
    }
    r.out.assign(n * (r.algo < 0 ? 32 : hb::digest_size(r.algo)), 0xEE);
    return r;
}

static int check_request(const Request &r, int status)
{
    if (r.cancelled) return status == HB_ECANCELED ? 0 : 1;
    if (status != HB_OK) {
        std::printf("request %llu failed with %d\n", (unsigned long long)r.ticket, status);
        return 1;
    }
    const uint32_t stride = r.algo < 0 ? 32u : uint32_t(hb::digest_size(r.algo));
    std::vector<uint8_t> want(stride);
    for (size_t i = 0; i < r.lens.size(); ++i) {
        const int a = r.algo < 0 ? r.algos[i] : r.algo;
        fingerprint(a, r.msgs.data() + r.offs[i], r.lens[i], want.data(), stride);
        if (std::memcmp(want.data(), r.out.data() + i * stride, stride) != 0) {
            std::printf("request %llu slot %zu: wrong digest\n", (unsigned long long)r.ticket, i);
            return 1;
        }
    }
    return 0;
}

int main(int argc, char **argv)
{
    const int clients = 3, per_client = argc > 1 ? std::atoi(argv[1]) : 60;
    hb_server *srv = nullptr;
    if (hb_server_create(&srv, 0, 2ull << 20, 48) != HB_OK) {
        std::printf("create failed: %s\n", hb_last_error());
        return 1;
    }
    std::atomic<int> bad{0}, done{0}, cancelled{0}, refused{0};
    std::vector<std::thread> th;
    for (int c = 0; c < clients; ++c)
        th.emplace_back([&, c] {
            std::mt19937_64 rng(1000 + c);
            std::vector<Request> reqs(per_client);
            for (int i = 0; i < per_client; ++i) {
                Request &r = reqs[i];
                r = make_request(rng);
                const int rc = hb_server_submit(srv, r.algo, r.algo < 0 ? r.algos.data() : nullptr, r.msgs.data(),
                                                r.offs.data(), r.lens.data(), r.lens.size(), r.out.data(), &r.ticket);
                if (rc == HB_EBUDGET) {  // a payload above the whole budget is refused at once
                    uint64_t total = 0;
                    for (uint64_t L : r.lens) total += L;
                    if (total <= (2ull << 20)) bad++;
                    r.ticket = 0;
                    refused++;
                    continue;
                }
                if (rc != HB_OK) {
                    std::printf("submit failed: %s\n", hb_last_error());
                    bad++;
                    continue;
                }
                if (rng() % 16 == 0 && hb_server_cancel(srv, r.ticket) == HB_OK) {
                    r.cancelled = true;
                    cancelled++;
                }
                // open-loop pacing with bursts: mostly back to back, sometimes a pause
                if (rng() % 8 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 3000));
            }
            for (Request &r : reqs) {
                if (!r.ticket) continue;
                int st = 0;
                if (hb_server_wait(srv, r.ticket, 120000, &st) != HB_OK) {
                    std::printf("wait failed: %s\n", hb_last_error());
                    bad++;
                    continue;
                }
                bad += check_request(r, st);
                done++;
                hb_server_release(srv, r.ticket);
            }
        });
    for (auto &t : th) t.join();
    uint64_t completed = 0, steps = 0, stalls = 0, peak = 0;
    hb_server_stats(srv, &completed, &steps, &stalls, &peak);
    hb_server_destroy(srv);
    const FakeHipReport rep = fake_hip_report();
    std::printf("requests %d (cancelled %d, refused over budget %d), steps %llu, admission stalls %llu, peak arena %llu B\n", int(done),
                int(cancelled), int(refused), (unsigned long long)steps, (unsigned long long)stalls, (unsigned long long)peak);
    std::printf("events created %ld destroyed %ld; most ops queued on one stream %ld; most events in flight %ld\n",
                rep.events_created, rep.events_destroyed, rep.max_ops_in_flight, rep.max_events_in_flight);
    std::printf("violations %ld%s%s; re-records in flight %ld; waits on unrecorded events %ld\n", rep.violations,
                rep.violations ? ": " : "", rep.first_violation.c_str(), rep.rerecords_in_flight, rep.waits_unrecorded);
    if (bad || rep.violations || rep.rerecords_in_flight || rep.waits_unrecorded ||
        rep.events_created != rep.events_destroyed || done + refused != clients * per_client) {
        std::printf("server check FAILED (bad %d)\n", int(bad));
        return 1;
    }
    std::printf("server ok\n");
    return 0;
}
