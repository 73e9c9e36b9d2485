// hb_server.cpp -- serving loop with continuous batching of hash requests.
//
// One background host thread owns the device side:
//   admission   requests leave the FIFO in arrival order while their payload fits the
//               device arena (the HBM budget) and a request slot is free;
//   staging     a pool of staging threads packs admitted requests -- a run of them whose
//               arena ranges follow each other at a time -- into a pinned ring per thread
//               and copies each run into the arena with one transfer, all on one copy
//               stream (one completion mark per run);
//   steps       staged requests are batched by class (only short chains / holding a long
//               one) into device steps on compute streams of their class (each with its
//               own plan), so a step can start while another is still hashing;
//   completion  a finished step's digests come back through pinned memory, each request
//               is marked done, and its arena range and slot are released.
// A request that arrives while others run is admitted as soon as memory and a slot free
// up, and its step overlaps the running ones on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/hb.h"
#include "hb_arena.hpp"
#include "hb_internal.hpp"
#include "hb_items.hpp"
#include "hb_outcome.hpp"
#include "hb_policy.hpp"
#include "hb_serve.hpp"
#include "hb_stage.hpp"

namespace hb {
namespace {

constexpr int kStreams = 8;                    // compute streams at most: 0 short requests,
                                               // the others long ones
constexpr int kLongStreamsDefault = 1;
constexpr uint64_t kLongChain = 128 * 1350;    // a request is "long" if its longest message's
                                               // chain exceeds this many ops (128 SM3 blocks)
constexpr size_t kMinBatch = 8;                // a step waits for this many staged requests...
constexpr double kMaxWait = 200e-6;            // ...or for its oldest request to wait this long (s),
                                               // unless no step is running
constexpr uint64_t kMaxStepN = 1ull << 20;     // messages per device step
constexpr int kMaxStagers = 16;                // staging threads at most
constexpr int kStagersDefault = 4;             // staging threads (HB_SERVER_STAGERS overrides)
constexpr uint64_t kPiece = 16ull << 20;       // largest single staging copy
constexpr uint64_t kRing = 64ull << 20;        // pinned staging ring per staging thread
constexpr size_t kMaxGroup = 256;              // requests staged together at most
constexpr size_t kMaxInflight = 64;            // copies in flight per staging thread at most
constexpr int kCopyStreams = 2;                // copy streams at most
// resident mode (HB_SERVER_MODE=resident): one resident launch takes published work items
constexpr uint64_t kResidentSlots = 1ull << 22;  // message slots (metadata and digest rings)
constexpr uint64_t kResidentItems = 1ull << 20;  // work-item ring entries (a power of two)
constexpr uint64_t kResidentIdleTicks = 500000;  // a launch ends 5 ms (100 MHz ticks) after its last item
constexpr uint64_t kResidentMaxTicks = 1000000000;  // and after 10 s in any case (the loop relaunches)

enum class St { Pending, Admitted, Launched, Done };

// Completion mark of one staged group's copies: an event recorded on the copy stream after
// the group's last piece, shared by the group's requests.
struct CopyMark {
    hipEvent_t ev = nullptr;
    int cs = 0;         // copy stream it was recorded on
    uint64_t seq = 0;   // position among the marks on that copy stream
    double t = -1;      // host time the serving loop first saw ev complete
    CopyMark() = default;
    CopyMark(const CopyMark &) = delete;
    CopyMark &operator=(const CopyMark &) = delete;
    ~CopyMark()
    {
        if (ev) hipEventDestroy(ev);
    }
};

struct Req {
    uint64_t ticket = 0;
    int algo = 0;                   // -1: per-message ids
    const uint8_t *algos = nullptr;
    const uint8_t *msgs = nullptr;
    const uint64_t *offs = nullptr, *lens = nullptr;
    uint64_t n = 0;
    uint8_t *out = nullptr;
    uint64_t payload = 0;           // sum of lengths
    uint64_t arena_off = Arena::kFail;
    St st = St::Pending;
    Outcome res;                    // status, and the text of a failure
    double t_submit = 0, t_admit = 0, t_h2d = 0, t_done = 0;
    double t_stage_begin = 0;       // host time a staging thread took it
    double t_staged = 0;            // host time its copies were enqueued
    double t_launch = 0;            // host time its step was launched
    double t_exec0 = 0, t_exec1 = 0;  // its step's inputs resident / digests back (host time the
                                      // loop saw the step's events complete)
    std::shared_ptr<CopyMark> copied;  // its staging group's copies
    bool stalled = false;           // was held back at the head of the queue
    int cls = 0;                    // 0: short chains only, 1: has a long chain
    // resident mode
    uint64_t slot0 = Arena::kFail;  // first of its n message slots
    std::vector<ServeItem> items;   // its work items (built by the staging thread)
    uint64_t item0 = 0;             // ring position of its first published item
    uint64_t checked = 0;           // items seen done so far
};

struct Step {
    std::vector<Req *> reqs;
    uint64_t n = 0;
    bool mixed = false;
    int algo = 0;
    hipEvent_t begin = nullptr;     // recorded when the step's inputs are resident
    hipEvent_t done = nullptr;
    double t_begin = -1;            // host time the loop first saw `begin` complete
};

// A staging thread's pinned ring.  Each copy occupies a segment of the ring until the copy
// completes; a new segment only waits for the oldest segments it would overwrite, so a
// slow copy holds back the thread only once the ring is full.
struct Segment {
    uint64_t begin, end;
    hipEvent_t copied;
};

struct Stager {
    std::thread thr;
    uint8_t *buf = nullptr;          // kRing pinned bytes
    uint8_t *dbuf = nullptr;         // their device mapping (kernel copies)
    int copy_stream = 0;             // index of the copy stream its transfers go on
    uint64_t head = 0;               // next free byte
    std::deque<Segment> inflight;    // in ring order, oldest first
    std::vector<hipEvent_t> spare;   // events of retired segments

    // Reserve `want` (<= kRing) contiguous bytes; returns their offset or kRing on error.
    // Also keeps fewer than kMaxInflight copies in flight: a ring of small requests would
    // otherwise queue thousands of transfers, and their events, on the copy stream.
    uint64_t reserve(uint64_t want)
    {
        head = (head + 255) & ~uint64_t(255);  // copies start 256-byte aligned
        if (head + want > kRing) head = 0;
        while (!inflight.empty()) {
            const Segment &o = inflight.front();
            const bool overlaps = !(o.end <= head || o.begin >= head + want);  // only the oldest can
            if (!overlaps && inflight.size() < kMaxInflight) break;
            if (hipEventSynchronize(o.copied) != hipSuccess) return kRing;
            spare.push_back(o.copied);
            inflight.pop_front();
        }
        return head;
    }
};
}  // namespace
}  // namespace hb

using namespace hb;

struct hb_server {
    int device = 0;
    uint64_t budget = 0;
    int max_slots = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    std::thread thr;
    std::deque<Req *> pending;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> all;
    uint64_t next_ticket = 1;
    int slots_used = 0;
    std::deque<Req *> to_stage;     // admitted, waiting for a staging thread (under mu)
    std::vector<Req *> staged[2];   // copies enqueued, waiting for a step, by class (under mu)
    std::condition_variable cv_stage;
    Stager stager[kMaxStagers];
    int n_stagers = kStagersDefault;
    bool stop_stagers = false;
    int staging_inflight = 0;       // requests a staging thread is working on (under mu)
    // owned by the loop thread
    Arena arena;
    uint8_t *d_arena = nullptr;
    std::vector<hipEvent_t> ev_pool;
    hipStream_t copy_in[kCopyStreams] = {};  // staging copies; staging thread w uses w % n_copy
    int n_copy = 1;
    bool copy_kernel = false;       // payload copies by kernel from the rings' device mapping
    std::mutex copy_mu[kCopyStreams];  // orders the copy marks' records on each copy stream
    uint64_t copy_seq[kCopyStreams] = {};  // (under copy_mu)
    // marks not yet seen complete, per copy stream in record order (under copy_mu): the
    // loop polls their heads and stamps each with the host time it first saw it done
    std::deque<std::shared_ptr<CopyMark>> unseen[kCopyStreams];
    hipStream_t compute[kStreams] = {};
    hb_plan *plan[kStreams][2] = {}; // per stream, by the class of the step it runs
    uint8_t *h_meta[kStreams] = {}; // pinned, coherent: offsets | lengths | ids | digests
    uint8_t *m_meta[kStreams] = {}; // the same buffer through its device mapping
    uint8_t *d_meta[kStreams] = {};
    std::unique_ptr<Step> busy[kStreams];
    int n_streams = kStreams;       // compute streams in use
    // resident mode: one launch of the serving kernel takes published work items; the rings
    // are pinned, coherent host memory the kernel reaches through its device mapping
    bool resident = false;
    ServeItem *r_items = nullptr;   // item ring (kResidentItems)
    uint64_t *r_ctl = nullptr;      // [0] items published (tail), [1] stop flag (low word)
    uint32_t *r_done = nullptr;     // per item ring entry: its position + 1 once hashed
    uint64_t *r_off = nullptr, *r_len = nullptr;  // per message slot
    uint32_t *r_slot = nullptr;     // per message slot: the caller's message index + slot0
    uint8_t *r_dig = nullptr;       // digest ring, 32 bytes per slot
    uint8_t *r_dev = nullptr;       // device: item ring copy, head, tail, stop
    ServeRings rings{};
    Arena slots;                    // message slots (owned by the loop thread)
    uint64_t published = 0;         // items published
    // items published and not yet seen done (written by the loop, read by the staging
    // threads to choose how to form a request's items)
    std::atomic<uint64_t> r_outstanding{0};
    uint64_t r_latency_items = 0;   // below this many outstanding items: latency formation
    uint32_t gen = 0;               // launches so far
    hipStream_t r_stream = nullptr;
    hipEvent_t r_ev = nullptr;      // recorded after each launch
    bool r_launched = false;
    int r_wgs = 0;                  // workgroups per launch
    std::vector<Req *> r_inflight;  // published, not finished
    int r_fail = HB_OK;             // set once a launch fails: every later request fails too
    std::string r_fail_why;
    std::chrono::steady_clock::time_point t0;
    // stats
    std::atomic<uint64_t> completed{0}, steps{0}, stalls{0}, peak{0};
    int fatal = HB_OK;

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace hb {
namespace {

constexpr uint64_t meta_bytes(uint64_t n) { return n * (8 + 8 + 1 + 32) + 1024; }

hipEvent_t take_event(hb_server *s)
{
    if (!s->ev_pool.empty()) {
        hipEvent_t e = s->ev_pool.back();
        s->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    return hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess ? e : nullptr;
}

// The text of the last error on this thread (set by set_error / hip_error).
std::string last_error_text() { return std::string(hb_last_error()); }

// Trace times are host times at which the loop saw a device event complete.  Every time
// on a request's trace is then on one clock (the server's steady clock), so the phases
// between them are never negative; each device time is late by at most one pass of the
// loop.  (Device timestamps mapped through one reference event drift against the host
// clock over a long run and carry the reference's own synchronisation latency.)
void poll_marks(hb_server *s)
{
    for (int c = 0; c < s->n_copy; ++c) {
        std::lock_guard<std::mutex> lk(s->copy_mu[c]);
        auto &q = s->unseen[c];
        while (!q.empty()) {
            const hipError_t e = hipEventQuery(q.front()->ev);
            if (e == hipErrorNotReady) break;  // later marks on this in-order stream are not done either
            q.front()->t = s->now();
            q.pop_front();
        }
    }
}

// Pack the group rs[0..k) (arena ranges following each other, see GroupPacker) into
// stager g's pinned ring and copy it into the arena on the copy stream, one copy per piece
// of at most kPiece bytes, so a group of small requests costs one transfer.  One mark
// recorded after the last piece is shared by the group's requests.
int stage_group(hb_server *s, Stager &g, Req *const *rs, int k)
{
    const int ci = g.copy_stream;
    hipStream_t cs = s->copy_in[ci];
    GroupPacker<Req> pk(rs, k);
    while (pk.done() < pk.total()) {
        const uint64_t want = std::min<uint64_t>(kPiece, pk.total() - pk.done());
        const uint64_t at = g.reserve(want);
        if (at == kRing) return set_error(HB_EHIP, "hb_server: staging wait");
        const uint64_t dst = pk.dst0() + pk.done();
        const uint64_t filled = pk.next(g.buf + at, want);
        if (filled != want) return set_error(HB_EINVAL, "hb_server: request shorter than its lengths");
        hipEvent_t ev = nullptr;
        if (!g.spare.empty()) {
            ev = g.spare.back();
            g.spare.pop_back();
        }
        hipError_t e = ev ? hipSuccess : hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess)
            e = s->copy_kernel ? launch_copy(s->d_arena + dst, g.dbuf + at, filled, cs)
                               : hipMemcpyAsync(s->d_arena + dst, g.buf + at, filled, hipMemcpyHostToDevice, cs);
        if (e == hipSuccess) e = hipEventRecord(ev, cs);
        if (e != hipSuccess) {
            if (ev) g.spare.push_back(ev);
            return hip_error(e, "hb_server: staging copy");
        }
        g.inflight.push_back({at, at + filled, ev});
        g.head = at + filled;
    }
    auto mark = std::make_shared<CopyMark>();
    hipError_t e = hipEventCreateWithFlags(&mark->ev, hipEventDisableTiming);
    if (e == hipSuccess) {
        std::lock_guard<std::mutex> lk(s->copy_mu[ci]);
        e = hipEventRecord(mark->ev, cs);
        if (e == hipSuccess) {
            mark->cs = ci;
            mark->seq = ++s->copy_seq[ci];
            s->unseen[ci].push_back(mark);
        }
    }
    if (e != hipSuccess) return hip_error(e, "hb_server: copy event");
    for (int q = 0; q < k; ++q) rs[q]->copied = mark;
    return HB_OK;
}

// Resident mode, on a staging thread: fill the request's message slots and build its work
// items (form_serve_items: slots by algorithm and block-count class, longest first; the
// latency formation while few items are outstanding).  Slot k holds the message's arena
// offset, length and the digest slot of its original index.
void prepare_items(hb_server *s, Req *r)
{
    const bool latency = s->r_outstanding.load(std::memory_order_relaxed) < s->r_latency_items;
    std::vector<uint32_t> slot_of;
    form_serve_items(
        r->n, r->lens, [&](uint64_t i) { return r->algo < 0 ? int(r->algos[i]) : r->algo; }, latency, slot_of,
        r->items);
    uint64_t pos = r->arena_off;
    for (uint64_t i = 0; i < r->n; ++i) {
        const uint64_t k = r->slot0 + slot_of[i];
        s->r_off[k] = pos;
        s->r_len[k] = r->lens[i];
        s->r_slot[k] = uint32_t(r->slot0 + i);
        pos += r->lens[i];
    }
    for (ServeItem &it : r->items) it.first += uint32_t(r->slot0);
}

// Staging thread: take admitted requests in order -- the head of the queue and the
// requests after it whose arena ranges continue it (up to the allocator's alignment), up
// to kPiece bytes -- stage them as one group and hand them to the loop.
void stager_loop(hb_server *s, int w)
{
    hipSetDevice(s->device);
    Stager &g = s->stager[w];
    std::vector<Req *> grp;
    for (;;) {
        grp.clear();
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_stage.wait(lk, [&] { return s->stop_stagers || !s->to_stage.empty(); });
            if (s->to_stage.empty()) return;
            uint64_t bytes = 0, next = 0;
            bool have = false;
            while (!s->to_stage.empty() && grp.size() < kMaxGroup) {
                Req *r = s->to_stage.front();
                if (r->payload) {
                    if (have && (r->arena_off != next || bytes + r->payload > kPiece)) break;
                    next = r->arena_off + Arena::round_up(r->payload);  // where the next range starts
                    have = true;
                    bytes += Arena::round_up(r->payload);
                }
                grp.push_back(r);
                s->to_stage.pop_front();
            }
            s->staging_inflight += int(grp.size());
            const double t0 = s->now();
            for (Req *r : grp) r->t_stage_begin = t0;
        }
        const int rc = stage_group(s, g, grp.data(), int(grp.size()));
        const std::string why = rc != HB_OK ? last_error_text() : std::string();
        if (rc == HB_OK && s->resident)
            for (Req *r : grp) prepare_items(s, r);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            const double t1 = s->now();
            for (Req *r : grp) {
                if (rc != HB_OK) r->res.fail(rc, why);
                r->t_staged = t1;
                s->staged[r->cls].push_back(r);
            }
            s->staging_inflight -= int(grp.size());
        }
        s->cv_work.notify_one();
    }
}

// Launch the staged requests of class c as one step on compute stream k.  Requests with
// only short chains are batched apart from those holding a long one, so a short request
// does not wait for another request's long chain to finish.
int launch_step(hb_server *s, int k, int c)
{
    auto st = std::make_unique<Step>();
    uint64_t n = 0;
    {
        std::lock_guard<std::mutex> g(s->mu);
        std::vector<Req *> &q = s->staged[c];
        size_t take = 0;
        while (take < q.size() && n + q[take]->n <= kMaxStepN) n += q[take++]->n;
        if (take == 0) return HB_OK;
        st->reqs.assign(q.begin(), q.begin() + take);
        q.erase(q.begin(), q.begin() + take);
        for (Req *r : st->reqs) r->st = St::Launched;
    }
    st->n = n;
    st->algo = st->reqs[0]->algo;
    for (Req *r : st->reqs) st->mixed |= (r->algo < 0 || r->algo != st->algo);
    const uint64_t stride = st->mixed ? 32 : uint64_t(digest_size(st->algo));
    // step metadata: absolute arena offsets, lengths, per-message ids
    uint64_t *ho = reinterpret_cast<uint64_t *>(s->h_meta[k]);
    uint64_t *hl = ho + kMaxStepN;
    uint8_t *hi = reinterpret_cast<uint8_t *>(hl + kMaxStepN);
    uint64_t m = 0;
    const CopyMark *last[kCopyStreams] = {};
    for (Req *r : st->reqs) {
        uint64_t pos = r->arena_off;
        for (uint64_t i = 0; i < r->n; ++i, ++m) {
            ho[m] = pos;
            hl[m] = r->lens[i];
            hi[m] = uint8_t(r->algo < 0 ? r->algos[i] : r->algo);
            pos += r->lens[i];
        }
        if (r->copied) {
            const CopyMark *&l = last[r->copied->cs];
            if (!l || r->copied->seq > l->seq) l = r->copied.get();
        }
    }
    // each copy stream is in order: once the step's latest mark on each is reached, every
    // copy the step reads has landed.  A failed wait fails the step: hashing arena bytes
    // whose copy has not landed would give wrong digests without an error.
    hipError_t we = hipSuccess;
    for (const CopyMark *l : last)
        if (l && we == hipSuccess) we = hipStreamWaitEvent(s->compute[k], l->ev, 0);
    {
        // trace times are read under the lock (hb_server_trace), so they are written under it
        std::lock_guard<std::mutex> g(s->mu);
        const double t_launch = s->now();
        for (Req *r : st->reqs) r->t_launch = t_launch;
    }
    uint64_t *dof = reinterpret_cast<uint64_t *>(s->d_meta[k]);
    uint64_t *dl = dof + kMaxStepN;
    uint8_t *di = reinterpret_cast<uint8_t *>(dl + kMaxStepN);
    uint8_t *dd = di + kMaxStepN;
    hipStream_t cs = s->compute[k];
    // on failure the step is parked on stream k with no event; the loop fails its requests
    auto fail = [&](int rc) {
        s->busy[k] = std::move(st);
        return rc;
    };
    if (we != hipSuccess) return fail(hip_error(we, "hb_server: step wait on its input copies"));
    // Metadata in and digests out are copied by kernels on the compute stream through the
    // pinned buffer's device mapping, not by the copy engine: a copy-engine transfer queued
    // behind a running step would hold up the payload copies of later requests.
    uint8_t *mm = s->m_meta[k];
    hipError_t e = launch_copy(dof, mm, n * 8, cs);
    if (e == hipSuccess) e = launch_copy(dl, mm + kMaxStepN * 8, n * 8, cs);
    if (e == hipSuccess && st->mixed) e = launch_copy(di, mm + kMaxStepN * 16, n, cs);
    if (e != hipSuccess) return fail(hip_error(e, "hb_server: step metadata"));
    st->begin = take_event(s);
    if (!st->begin || hipEventRecord(st->begin, cs) != hipSuccess) return fail(set_error(HB_EHIP, "hb_server: step event"));
    int rc = hb_plan_run(s->plan[k][c], st->mixed ? di : nullptr, st->algo, s->d_arena, dof, dl, n, dd, cs);
    if (rc != HB_OK) return fail(rc);
    e = launch_copy(mm + kMaxStepN * 17, dd, n * stride, cs);
    if (e != hipSuccess) return fail(hip_error(e, "hb_server: digest copy"));
    hipEvent_t done = take_event(s);
    if (!done || hipEventRecord(done, cs) != hipSuccess) {
        if (done) s->ev_pool.push_back(done);
        return fail(set_error(HB_EHIP, "hb_server: step event"));
    }
    st->done = done;
    s->busy[k] = std::move(st);
    s->steps++;
    return HB_OK;
}

// Finish the step on stream k: digests to the callers' buffers, release memory and slots.
// A failed step (status != HB_OK) fails each of its requests with `why`.
void finish_step(hb_server *s, int k, int status, const std::string &why)
{
    Step *st = s->busy[k].get();
    const uint64_t stride = st->mixed ? 32 : uint64_t(digest_size(st->algo));
    const uint8_t *hd = s->h_meta[k] + kMaxStepN * 17;
    poll_marks(s);  // every mark the step waited on is complete if the step is
    const double t = s->now();
    const double t_exec0 = st->t_begin >= 0 ? st->t_begin : t;
    // digests first; a request's status, trace times and state change together under the
    // lock, where hb_server_wait / poll / trace read them
    std::vector<double> t_h2d(st->reqs.size());
    uint64_t m = 0;
    for (size_t q = 0; q < st->reqs.size(); ++q) {
        Req *r = st->reqs[q];
        const uint64_t ds = r->algo < 0 ? 32 : uint64_t(digest_size(r->algo));
        if (status == HB_OK && r->res.status == HB_OK) {  // res is only written under the lock
            if (ds == stride) std::memcpy(r->out, hd + m * stride, r->n * stride);
            else
                for (uint64_t i = 0; i < r->n; ++i) std::memcpy(r->out + i * ds, hd + (m + i) * stride, ds);
        }
        m += r->n;
        if (r->copied) {
            const CopyMark &c = *r->copied;
            t_h2d[q] = c.t >= 0 ? std::min(c.t, t_exec0) : t_exec0;
            r->copied.reset();
        } else {
            t_h2d[q] = -1;  // nothing to copy: the time its staging ended
        }
        if (r->payload) s->arena.release(r->arena_off, r->payload);
    }
    if (st->begin) s->ev_pool.push_back(st->begin);
    if (st->done) s->ev_pool.push_back(st->done);
    {
        std::lock_guard<std::mutex> g(s->mu);
        for (size_t q = 0; q < st->reqs.size(); ++q) {
            Req *r = st->reqs[q];
            r->res.fail(status, why);
            r->t_exec0 = t_exec0;
            r->t_exec1 = t;
            r->t_h2d = t_h2d[q] >= 0 ? t_h2d[q] : r->t_staged;
            r->t_done = t;
            r->st = St::Done;
            s->slots_used--;
        }
    }
    s->completed += st->reqs.size();
    s->busy[k].reset();
    s->cv_done.notify_all();
}

// Resident mode: publish the work items of staged requests whose payload has landed (their
// copy mark seen complete), in staging order, while the item ring has room.
int resident_publish(hb_server *s)
{
    std::vector<Req *> ready;
    {
        std::lock_guard<std::mutex> g(s->mu);
        for (int c = 0; c < 2; ++c) {
            std::vector<Req *> &q = s->staged[c];
            size_t keep = 0;
            for (size_t i = 0; i < q.size(); ++i) {
                Req *r = q[i];
                const bool landed = !r->copied || r->copied->t >= 0 || r->res.status != HB_OK;
                if (landed) {
                    r->st = St::Launched;
                    ready.push_back(r);
                } else {
                    q[keep++] = r;
                }
            }
            q.resize(keep);
        }
    }
    if (ready.empty()) return 0;
    const uint64_t mask = kResidentItems - 1;
    uint64_t oldest = s->published;
    for (Req *r : s->r_inflight) oldest = std::min(oldest, r->item0 + r->checked);
    const double t = s->now();
    std::vector<Req *> failed;
    for (Req *r : ready) {
        if (r->res.status != HB_OK) {  // staging failed: nothing to hash
            failed.push_back(r);
            continue;
        }
        // the ring never holds more than kResidentItems unfinished items (it has far more
        // room than max_slots requests of 2^20 messages need: 16,384 items each at most)
        while (s->published + r->items.size() - oldest > kResidentItems) {
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            oldest = s->published;
            for (Req *q : s->r_inflight) {
                while (q->checked < q->items.size()) {
                    const uint64_t h = q->item0 + q->checked;
                    if (__atomic_load_n(&s->r_done[h & mask], __ATOMIC_ACQUIRE) != uint32_t(h + 1)) break;
                    q->checked++;
                    s->r_outstanding.fetch_sub(1, std::memory_order_relaxed);
                }
                oldest = std::min(oldest, q->item0 + q->checked);
            }
        }
        r->item0 = s->published;
        r->checked = 0;
        for (size_t k = 0; k < r->items.size(); ++k) s->r_items[(s->published + k) & mask] = r->items[k];
        s->published += r->items.size();
        s->r_outstanding.fetch_add(r->items.size(), std::memory_order_relaxed);
        s->r_inflight.push_back(r);
    }
    __atomic_store_n(&s->r_ctl[0], s->published, __ATOMIC_RELEASE);
    {
        std::lock_guard<std::mutex> g(s->mu);
        for (Req *r : ready) {
            r->t_launch = t;
            r->t_exec0 = t;
        }
    }
    for (Req *r : failed) {  // no items: finishes at once with its staging failure
        if (r->payload) s->arena.release(r->arena_off, r->payload);
        s->slots.release(r->slot0, r->n);
        std::lock_guard<std::mutex> g(s->mu);
        r->t_h2d = r->t_exec1 = r->t_done = t;
        r->st = St::Done;
        s->slots_used--;
    }
    if (!failed.empty()) s->cv_done.notify_all();
    return int(ready.size());
}

// Resident mode: finish the published requests whose items are all done (their digests
// to the callers' buffers, memory and slots released), fail them all if the launch failed,
// and relaunch the serving kernel when items wait and no launch is running.  Returns the
// number of requests finished.
int resident_progress(hb_server *s)
{
    const uint64_t mask = kResidentItems - 1;
    bool running = false;
    if (s->r_launched) {
        const hipError_t q = hipEventQuery(s->r_ev);
        if (q == hipErrorNotReady) running = true;
        else if (q != hipSuccess && s->r_fail == HB_OK) {
            s->r_fail = HB_EHIP;
            s->r_fail_why = std::string("hb_server: serving kernel failed on the device: ") + hipGetErrorString(q);
        }
        if (!running) s->r_launched = false;
    }
    const int fail = s->r_fail;
    const std::string why = s->r_fail_why;
    poll_marks(s);
    const double t = s->now();
    int finished = 0;
    size_t keep = 0;
    for (size_t i = 0; i < s->r_inflight.size(); ++i) {
        Req *r = s->r_inflight[i];
        const uint64_t checked0 = r->checked;
        while (fail == HB_OK && r->checked < r->items.size()) {
            const uint64_t h = r->item0 + r->checked;
            if (__atomic_load_n(&s->r_done[h & mask], __ATOMIC_ACQUIRE) != uint32_t(h + 1)) break;
            r->checked++;
        }
        if (fail == HB_OK && r->checked < r->items.size()) {
            s->r_outstanding.fetch_sub(r->checked - checked0, std::memory_order_relaxed);
            s->r_inflight[keep++] = r;
            continue;
        }
        s->r_outstanding.fetch_sub(r->items.size() - checked0, std::memory_order_relaxed);  // the rest, on failure too
        const uint64_t ds = r->algo < 0 ? 32 : uint64_t(digest_size(r->algo));
        if (fail == HB_OK) {
            // slot k holds the digest of message r_slot[k] - slot0 (slots are in item order)
            for (uint64_t k = r->slot0; k < r->slot0 + r->n; ++k)
                std::memcpy(r->out + (s->r_slot[k] - r->slot0) * ds, s->r_dig + k * 32, ds);
        }
        const double h2d = r->copied ? (r->copied->t >= 0 ? std::min(r->copied->t, r->t_exec0) : r->t_exec0) : -1;
        r->copied.reset();
        if (r->payload) s->arena.release(r->arena_off, r->payload);
        s->slots.release(r->slot0, r->n);
        {
            std::lock_guard<std::mutex> g(s->mu);
            r->res.fail(fail, why);
            r->t_h2d = h2d >= 0 ? h2d : r->t_staged;
            r->t_exec1 = t;
            r->t_done = t;
            r->st = St::Done;
            s->slots_used--;
        }
        ++finished;
    }
    s->r_inflight.resize(keep);
    if (finished) {
        s->completed += uint64_t(finished);
        s->cv_done.notify_all();
    }
    if (!s->r_inflight.empty() && !running && s->r_fail == HB_OK) {
        // items wait and no launch takes them: start one (head and tail persist on the
        // device, so it picks up whatever the last launch left)
        const hipError_t e = launch_serve(s->rings, ++s->gen, s->r_wgs, s->r_stream);
        const hipError_t er = e == hipSuccess ? hipEventRecord(s->r_ev, s->r_stream) : e;
        if (er != hipSuccess) {
            s->fatal = HB_EHIP;
            s->r_fail = HB_EHIP;
            s->r_fail_why = std::string("hb_server: serving kernel launch: ") + hipGetErrorString(er);
        } else {
            s->r_launched = true;
            s->steps++;
        }
    }
    return finished;
}

void loop(hb_server *s)
{
    hipSetDevice(s->device);
    for (;;) {
        // 1. admission, in arrival order; admitted requests go to the staging threads
        size_t admitted = 0;
        int launch_cls[kStreams];  // class to launch on each idle stream
        std::fill(launch_cls, launch_cls + kStreams, -1);
        {
            std::unique_lock<std::mutex> g(s->mu);
            bool any_busy = !s->r_inflight.empty();
            for (auto &b : s->busy) any_busy |= bool(b);
            if (s->pending.empty() && s->to_stage.empty() && s->staging_inflight == 0 && s->staged[0].empty() &&
                s->staged[1].empty() && !any_busy) {
                if (s->stop) break;
                s->cv_work.wait_for(g, std::chrono::milliseconds(50));
                continue;
            }
            admitted = admit_in_order(
                s->pending, s->arena, s->slots_used, s->max_slots,
                [&](Req *r) {
                    r->st = St::Admitted;
                    r->t_admit = s->now();
                    s->to_stage.push_back(r);
                },
                [&](Req *r) {  // resident mode: message slots too
                    if (!s->resident) return true;
                    const uint64_t o = s->slots.alloc(r->n);
                    if (o == Arena::kFail) return false;
                    r->slot0 = o;
                    return true;
                });
            if (!s->pending.empty() && !s->pending.front()->stalled) {
                s->pending.front()->stalled = true;
                s->stalls++;
            }
            if (s->arena.peak() > s->peak) s->peak = s->arena.peak();
            // continuous batching (choose_launches): one step per class at a time, on an
            // idle stream of its class, once enough requests are staged or the oldest has
            // waited long enough; an idle stream may take the other class's step
            LaunchInputs in;
            bool busy[kStreams];
            for (int k = 0; k < s->n_streams; ++k) busy[k] = bool(s->busy[k]);
            in.n_streams = s->n_streams;
            in.busy = busy;
            for (int c = 0; c < 2; ++c) {
                in.staged[c] = s->staged[c].size();
                in.oldest_staged[c] = s->staged[c].empty() ? 0.0 : s->staged[c].front()->t_staged;
            }
            in.now = s->now();
            in.min_batch = kMinBatch;
            in.max_wait = kMaxWait;
            if (!s->resident) choose_launches(in, launch_cls);
        }
        if (admitted) s->cv_stage.notify_all();
        if (s->resident) {
            // resident mode: requests join the running launch as soon as their payload lands
            poll_marks(s);
            const int published = resident_publish(s);
            const int finished = resident_progress(s);
            if (!published && !finished && !admitted) std::this_thread::sleep_for(std::chrono::microseconds(10));
            continue;
        }
        // 2. launch steps on idle compute streams
        for (int k = 0; k < s->n_streams; ++k) {
            if (launch_cls[k] < 0) continue;
            int rc = launch_step(s, k, launch_cls[k]);
            if (rc != HB_OK) {
                std::string why = last_error_text();
                s->fatal = rc;
                if (s->busy[k]) {
                    const hipError_t e = hipStreamSynchronize(s->compute[k]);
                    if (e != hipSuccess) {
                        rc = HB_EHIP;
                        why += std::string("; stream: ") + hipGetErrorString(e);
                    }
                    finish_step(s, k, rc, why);
                }
            }
        }
        // 3. completions: input copies seen done, steps begun, steps done (in this order, so
        // a request's trace times never run backwards)
        poll_marks(s);
        bool progressed = false;
        for (int k = 0; k < s->n_streams; ++k) {
            Step *st = s->busy[k].get();
            if (!st) continue;
            if (st->t_begin < 0 && st->begin && hipEventQuery(st->begin) == hipSuccess) st->t_begin = s->now();
            const hipError_t q = hipEventQuery(st->done);
            if (q == hipSuccess) { finish_step(s, k, HB_OK, std::string()); progressed = true; }
            else if (q != hipErrorNotReady) {
                finish_step(s, k, HB_EHIP, std::string("hb_server: step failed on the device: ") + hipGetErrorString(q));
                progressed = true;
            }
        }
        if (!progressed && !admitted) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

}  // namespace
}  // namespace hb

extern "C" {

int hb_server_create(hb_server **out, int device, uint64_t hbm_budget_bytes, int max_slots)
{
    if (!out) return set_error(HB_EINVAL, "hb_server_create: null server pointer");
    *out = nullptr;
    if (hbm_budget_bytes < Arena::kAlign || max_slots <= 0)
        return set_error(HB_EINVAL, "hb_server_create: budget must be >= 256 bytes and max_slots > 0");
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return hip_error(e, "hb_server_create: hipSetDevice");
    auto s = std::make_unique<hb_server>();
    s->device = device;
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    s->t0 = std::chrono::steady_clock::now();
    s->arena.reset(hbm_budget_bytes);
    auto fail = [&](int rc, const char *what, hipError_t he) {
        // partial resources are released by the destructor path below
        hb_server *p = s.release();
        p->stop = true;
        hb_server_destroy(p);
        return he != hipSuccess ? hip_error(he, what) : set_error(rc, what);
    };
    if ((e = hipMalloc(reinterpret_cast<void **>(&s->d_arena), s->arena.capacity())) != hipSuccess)
        return fail(HB_ENOMEM, "hb_server_create: device arena", hipSuccess);
    if (const char *v = std::getenv("HB_SERVER_STAGERS")) s->n_stagers = std::max(1, std::min(kMaxStagers, std::atoi(v)));
    if (const char *v = std::getenv("HB_SERVER_COPY")) s->copy_kernel = std::strcmp(v, "kernel") == 0;
    for (int w = 0; w < s->n_stagers; ++w) {
        const unsigned fl = s->copy_kernel ? (hipHostMallocMapped | hipHostMallocCoherent) : hipHostMallocDefault;
        if ((e = hipHostMalloc(reinterpret_cast<void **>(&s->stager[w].buf), kRing, fl)) != hipSuccess)
            return fail(HB_ENOMEM, "hb_server_create: pinned staging", hipSuccess);
        if (s->copy_kernel &&
            (e = hipHostGetDevicePointer(reinterpret_cast<void **>(&s->stager[w].dbuf), s->stager[w].buf, 0)) != hipSuccess)
            return fail(HB_EHIP, "hb_server_create: device mapping of staging", e);
    }
    // copy streams: two when the process has eight hardware queues (two copy engines at
    // work), else one; HB_SERVER_COPY_STREAMS overrides
    if (const char *v = std::getenv("GPU_MAX_HW_QUEUES"); v && std::atoi(v) >= 8) s->n_copy = 2;
    if (const char *v = std::getenv("HB_SERVER_COPY_STREAMS")) s->n_copy = std::max(1, std::min(kCopyStreams, std::atoi(v)));
    for (int c = 0; c < s->n_copy; ++c)
        if ((e = hipStreamCreateWithFlags(&s->copy_in[c], hipStreamNonBlocking)) != hipSuccess)
            return fail(HB_EHIP, "hb_server_create: stream", e);
    for (int w = 0; w < s->n_stagers; ++w) s->stager[w].copy_stream = w % s->n_copy;
    // Compute streams: one for short-chain steps, kLongStreamsDefault for long-chain ones,
    // two when the process has eight hardware queues (HB_SERVER_LONG_STREAMS overrides,
    // up to kStreams - 1).  Every stream may take one of the process's hardware queues
    // (HIP's default is four, and the application's own default stream holds one once
    // used); streams sharing a queue wait behind each other's kernels, and a copy stream
    // sharing one with a compute stream stalls every request behind multi-millisecond
    // chains.  So with four queues the loop keeps to three streams (copy, short, long),
    // with eight to five (two copy, two long), and its plans take no side stream.  Each
    // stream keeps a plan per step
    // class, since an idle stream also runs the other class's steps: short-chain steps
    // are plain persistent-kernel plans (nothing in them reaches the long-chain
    // threshold); long-chain steps take the long-chain path in one launch with the bulk
    // (HB_PLAN_LONG_INLINE), so their longest chains run rounds-only from precomputed
    // schedule words beside the bulk -- the chain is what such a step's latency is.
    // HB_SERVER_LONG_PLAN_FLAGS sets the long-chain plans' flags, HB_SERVER_PLAN_FLAGS
    // every plan's.  Plans launch eagerly.
    if (const char *v = std::getenv("HB_SERVER_MODE")) s->resident = std::strcmp(v, "resident") == 0;
    if (s->resident) {
        // resident mode: the rings (pinned, coherent, mapped), the device copy of the item
        // ring with its head, tail and stop words, one stream for the serving launches
        const unsigned fl = hipHostMallocMapped | hipHostMallocCoherent;
        auto pinned = [&](void **p, uint64_t bytes) { return hipHostMalloc(p, bytes, fl); };
        if ((e = pinned(reinterpret_cast<void **>(&s->r_items), kResidentItems * sizeof(ServeItem))) != hipSuccess ||
            (e = pinned(reinterpret_cast<void **>(&s->r_ctl), 256)) != hipSuccess ||
            (e = pinned(reinterpret_cast<void **>(&s->r_done), kResidentItems * 4)) != hipSuccess ||
            (e = pinned(reinterpret_cast<void **>(&s->r_off), kResidentSlots * 8)) != hipSuccess ||
            (e = pinned(reinterpret_cast<void **>(&s->r_len), kResidentSlots * 8)) != hipSuccess ||
            (e = pinned(reinterpret_cast<void **>(&s->r_slot), kResidentSlots * 4)) != hipSuccess ||
            (e = pinned(reinterpret_cast<void **>(&s->r_dig), kResidentSlots * 32)) != hipSuccess)
            return fail(HB_ENOMEM, "hb_server_create: pinned serving rings", hipSuccess);
        std::memset(s->r_ctl, 0, 256);
        std::memset(s->r_done, 0, kResidentItems * 4);
        const uint64_t dev_bytes = kResidentItems * sizeof(ServeItem) + 256;
        if ((e = hipMalloc(reinterpret_cast<void **>(&s->r_dev), dev_bytes)) != hipSuccess)
            return fail(HB_ENOMEM, "hb_server_create: device item ring", hipSuccess);
        if ((e = hipMemset(s->r_dev + kResidentItems * sizeof(ServeItem), 0, 256)) != hipSuccess)
            return fail(HB_EHIP, "hb_server_create: device ring words", e);
        ServeRings &R = s->rings;
        void *m = nullptr;
        auto map = [&](void *h) {
            return hipHostGetDevicePointer(&m, h, 0) == hipSuccess ? m : nullptr;
        };
        R.h_items = static_cast<const ServeItem *>(map(s->r_items));
        R.h_tail = static_cast<const uint64_t *>(map(s->r_ctl));
        R.h_stop = reinterpret_cast<const uint32_t *>(R.h_tail ? R.h_tail + 1 : nullptr);
        R.done = static_cast<uint32_t *>(map(s->r_done));
        R.off = static_cast<const uint64_t *>(map(s->r_off));
        R.len = static_cast<const uint64_t *>(map(s->r_len));
        R.digests = static_cast<uint8_t *>(map(s->r_dig));
        if (!R.h_items || !R.h_tail || !R.done || !R.off || !R.len || !R.digests)
            return fail(HB_EHIP, "hb_server_create: device mapping of serving rings", hipErrorInvalidValue);
        R.arena = s->d_arena;
        R.d_items = reinterpret_cast<ServeItem *>(s->r_dev);
        uint64_t *words = reinterpret_cast<uint64_t *>(s->r_dev + kResidentItems * sizeof(ServeItem));
        R.d_head = words;
        R.d_tail = words + 1;
        R.d_stop = reinterpret_cast<uint32_t *>(words + 2);
        R.items_cap = kResidentItems;
        R.idle_ticks = kResidentIdleTicks;
        if (const char *v = std::getenv("HB_SERVER_RESIDENT_IDLE_MS"))  // 100 MHz ticks per ms
            R.idle_ticks = uint64_t(std::max(1, std::min(60000, std::atoi(v)))) * 100000ull;
        R.max_ticks = kResidentMaxTicks;
        s->slots.reset(kResidentSlots);
        int cus = 0;
        if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device)) != hipSuccess)
            return fail(HB_EHIP, "hb_server_create: CU count", e);
        // one workgroup (four waves) on every other CU: the payload copies run as kernels
        // on the copy streams, and with a serving workgroup on every CU their completion
        // trailed by milliseconds at high load (copy p99 4.5-16.6 ms from 0.5 to 0.9 of
        // capacity, against 0.2-1.2 ms, and a higher capacity, with half the CUs)
        s->r_wgs = std::max(cus / 2, 1);
        if (const char *v = std::getenv("HB_SERVER_RESIDENT_WGS")) s->r_wgs = std::max(1, std::min(65536, std::atoi(v)));
        // latency formation while fewer items are outstanding than twice the launch's waves.
        // On the serving mix (requests of 1..10,000 messages, log-normal lengths capped at
        // 64 KiB) a cooperative item costs little wave time -- about 1 % of the messages
        // reach 128 blocks -- and it shortens the longest chain, which is a request's
        // latency: p99 at 0.7 of capacity 3.55 ms with half the worker waves as the limit,
        // 2.66 ms with twice, 2.72 ms with no limit, capacity within 1 % of each other
        s->r_latency_items = uint64_t(s->r_wgs) * (kServeThreads / 64) * 2;
        if (const char *v = std::getenv("HB_SERVER_RESIDENT_LATENCY_ITEMS")) s->r_latency_items = uint64_t(std::max(0, std::atoi(v)));
        if ((e = hipStreamCreateWithFlags(&s->r_stream, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&s->r_ev, hipEventDisableTiming)) != hipSuccess)
            return fail(HB_EHIP, "hb_server_create: serving stream", e);
        s->n_streams = 0;
        hb_server *p = s.release();
        for (int w = 0; w < p->n_stagers; ++w) p->stager[w].thr = std::thread(stager_loop, p, w);
        p->thr = std::thread(loop, p);
        *out = p;
        return HB_OK;
    }
    int n_long = kLongStreamsDefault;
    // a process started with GPU_MAX_HW_QUEUES >= 8 (HIP's hardware queues per process)
    // has queues for a second long-chain stream
    if (const char *v = std::getenv("GPU_MAX_HW_QUEUES"); v && std::atoi(v) >= 8) n_long = 2;
    if (const char *v = std::getenv("HB_SERVER_LONG_STREAMS")) n_long = std::max(1, std::min(kStreams - 1, std::atoi(v)));
    s->n_streams = 1 + n_long;
    int plan_flags[2] = {HB_PLAN_NO_LONG, HB_PLAN_LONG_INLINE};  // by step class
    if (const char *v = std::getenv("HB_SERVER_PLAN_FLAGS")) plan_flags[0] = plan_flags[1] = std::atoi(v);
    if (const char *v = std::getenv("HB_SERVER_LONG_PLAN_FLAGS")) plan_flags[1] = std::atoi(v);
    for (int k = 0; k < s->n_streams; ++k) {
        if ((e = hipStreamCreateWithFlags(&s->compute[k], hipStreamNonBlocking)) != hipSuccess)
            return fail(HB_EHIP, "hb_server_create: stream", e);
        for (int c = 0; c < 2; ++c) {
            int rc = hb_plan_create(&s->plan[k][c], kMaxStepN, plan_flags[c]);
            if (rc != HB_OK) return fail(rc, "hb_server_create: plan", hipSuccess);
        }
        if ((e = hipHostMalloc(reinterpret_cast<void **>(&s->h_meta[k]), meta_bytes(kMaxStepN),
                               hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess)
            return fail(HB_ENOMEM, "hb_server_create: pinned step buffers", hipSuccess);
        if ((e = hipHostGetDevicePointer(reinterpret_cast<void **>(&s->m_meta[k]), s->h_meta[k], 0)) != hipSuccess)
            return fail(HB_EHIP, "hb_server_create: device mapping of step buffers", e);
        if ((e = hipMalloc(reinterpret_cast<void **>(&s->d_meta[k]), meta_bytes(kMaxStepN))) != hipSuccess)
            return fail(HB_ENOMEM, "hb_server_create: device step buffers", hipSuccess);
    }
    hb_server *p = s.release();
    for (int w = 0; w < p->n_stagers; ++w) p->stager[w].thr = std::thread(stager_loop, p, w);
    p->thr = std::thread(loop, p);
    *out = p;
    return HB_OK;
}

int hb_server_submit(hb_server *s, int algo_or_mixed, const uint8_t *algos, const uint8_t *messages,
                     const uint64_t *offsets, const uint64_t *lengths, uint64_t n, uint8_t *digests_out,
                     uint64_t *ticket)
{
    if (!s || !ticket) return set_error(HB_EINVAL, "hb_server_submit: null server or ticket pointer");
    const bool mixed = algo_or_mixed == -1;
    if (!mixed && digest_size(algo_or_mixed) == 0) return set_error(HB_EINVAL, "hb_server_submit: unknown algorithm id");
    if (n == 0) return set_error(HB_EINVAL, "hb_server_submit: empty request");
    if (n > kMaxStepN) return set_error(HB_EINVAL, "hb_server_submit: more than 2^20 messages in one request");
    if (!offsets || !lengths || !digests_out || (mixed && !algos))
        return set_error(HB_EINVAL, "hb_server_submit: null host pointer");
    uint64_t payload = 0, chain = 0;
    static constexpr uint64_t kOps[3] = {340, 620, 1350};  // VALU ops per block
    for (uint64_t i = 0; i < n; ++i) {
        if (lengths[i] >= (1ull << 61)) return set_error(HB_EINVAL, "hb_server_submit: length beyond 2^61");
        if (mixed && algos[i] > HB_SM3) return set_error(HB_EINVAL, "hb_server_submit: unknown algorithm id in algos");
        payload += lengths[i];
        const uint64_t c = ((lengths[i] + 8) / 64 + 1) * kOps[mixed ? algos[i] : algo_or_mixed];
        chain = c > chain ? c : chain;
    }
    if (payload && !messages) return set_error(HB_EINVAL, "hb_server_submit: null messages");
    if (Arena::round_up(payload) > s->arena.capacity())
        return set_error(HB_EBUDGET, "hb_server_submit: request payload exceeds the device budget");
    auto r = std::make_unique<Req>();
    r->algo = mixed ? -1 : algo_or_mixed;
    r->algos = algos;
    r->msgs = messages;
    r->offs = offsets;
    r->lens = lengths;
    r->n = n;
    r->out = digests_out;
    r->payload = payload;
    r->cls = chain > kLongChain ? 1 : 0;
    r->t_submit = s->now();
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) return set_error(HB_EINVAL, "hb_server_submit: server is stopping");
        r->ticket = s->next_ticket++;
        *ticket = r->ticket;
        s->pending.push_back(r.get());
        s->all[r->ticket] = std::move(r);
    }
    s->cv_work.notify_one();
    return HB_OK;
}

int hb_server_poll(hb_server *s, uint64_t ticket, int *done, int *status)
{
    if (!s || !done) return set_error(HB_EINVAL, "hb_server_poll: null pointer");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return set_error(HB_EINVAL, "hb_server_poll: unknown ticket");
    *done = it->second->st == St::Done;
    if (status) *status = it->second->res.status;
    // a failed request's explanation becomes this thread's last error
    if (*done) it->second->res.deliver([](int st, const std::string &why) { set_error(st, why); });
    return HB_OK;
}

int hb_server_cancel(hb_server *s, uint64_t ticket)
{
    if (!s) return set_error(HB_EINVAL, "hb_server_cancel: null server");
    {
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->all.find(ticket);
        if (it == s->all.end()) return set_error(HB_EINVAL, "hb_server_cancel: unknown ticket");
        Req *r = it->second.get();
        if (r->st != St::Pending) return set_error(HB_EBUSY, "hb_server_cancel: request already admitted");
        auto q = std::find(s->pending.begin(), s->pending.end(), r);
        if (q == s->pending.end()) return set_error(HB_EBUSY, "hb_server_cancel: request already admitted");
        s->pending.erase(q);
        r->res.fail(HB_ECANCELED, "hb_server_cancel: cancelled before admission");
        r->t_admit = r->t_h2d = r->t_done = s->now();
        r->st = St::Done;
    }
    s->cv_done.notify_all();
    s->cv_work.notify_one();  // the next request may now be admissible
    return HB_OK;
}

int hb_server_release(hb_server *s, uint64_t ticket)
{
    if (!s) return set_error(HB_EINVAL, "hb_server_release: null server");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return set_error(HB_EINVAL, "hb_server_release: unknown ticket");
    if (it->second->st != St::Done) return set_error(HB_EBUSY, "hb_server_release: request not finished");
    s->all.erase(it);
    return HB_OK;
}

int hb_server_wait(hb_server *s, uint64_t ticket, int64_t timeout_ms, int *status)
{
    if (!s) return set_error(HB_EINVAL, "hb_server_wait: null server");
    std::unique_lock<std::mutex> g(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return set_error(HB_EINVAL, "hb_server_wait: unknown ticket");
    Req *r = it->second.get();
    auto ready = [&] { return r->st == St::Done; };
    if (timeout_ms < 0) s->cv_done.wait(g, ready);
    else if (!s->cv_done.wait_for(g, std::chrono::milliseconds(timeout_ms), ready))
        return set_error(HB_EBUSY, "hb_server_wait: timed out");
    if (status) *status = r->res.status;
    // a failed request's explanation becomes this thread's last error
    r->res.deliver([](int st, const std::string &why) { set_error(st, why); });
    return HB_OK;
}

int hb_server_times(hb_server *s, uint64_t ticket, double *t_submit, double *t_admit, double *t_h2d_done,
                    double *t_done)
{
    if (!s) return set_error(HB_EINVAL, "hb_server_times: null server");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return set_error(HB_EINVAL, "hb_server_times: unknown ticket");
    Req *r = it->second.get();
    if (t_submit) *t_submit = r->t_submit;
    if (t_admit) *t_admit = r->t_admit;
    if (t_h2d_done) *t_h2d_done = r->t_h2d;
    if (t_done) *t_done = r->t_done;
    return HB_OK;
}

int hb_server_trace(hb_server *s, uint64_t ticket, double *t, int nt)
{
    if (!s) return set_error(HB_EINVAL, "hb_server_trace: null server");
    if (nt < 0 || (nt > 0 && !t)) return set_error(HB_EINVAL, "hb_server_trace: null or negative-size output");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return set_error(HB_EINVAL, "hb_server_trace: unknown ticket");
    const Req *r = it->second.get();
    const double v[HB_TRACE_COUNT] = {r->t_submit, r->t_admit, r->t_stage_begin, r->t_staged, r->t_h2d,
                                      r->t_launch, r->t_exec0,  r->t_exec1,        r->t_done};
    for (int i = 0; i < nt && i < HB_TRACE_COUNT; ++i) t[i] = v[i];
    for (int i = HB_TRACE_COUNT; i < nt; ++i) t[i] = 0.0;
    return HB_OK;
}

int hb_server_stats(hb_server *s, uint64_t *completed, uint64_t *nsteps, uint64_t *stalls, uint64_t *peak_bytes)
{
    if (!s) return set_error(HB_EINVAL, "hb_server_stats: null server");
    if (completed) *completed = s->completed;
    if (nsteps) *nsteps = s->steps;
    if (stalls) *stalls = s->stalls;
    if (peak_bytes) *peak_bytes = s->peak;
    return HB_OK;
}

double hb_server_now(hb_server *s) { return s ? s->now() : 0.0; }

void hb_server_destroy(hb_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->thr.joinable()) s->thr.join();
    // resident mode: the host's stop flag ends the serving kernel's wait for items at once
    // (it would otherwise stay up to its idle limit); it must be gone before any free below,
    // since freeing memory waits for the device's work to finish
    if (s->r_ctl) __atomic_store_n(reinterpret_cast<uint32_t *>(s->r_ctl + 1), 1u, __ATOMIC_RELEASE);
    if (s->r_stream) hipStreamSynchronize(s->r_stream);
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop_stagers = true;
    }
    s->cv_stage.notify_all();
    for (Stager &g : s->stager) {
        if (g.thr.joinable()) g.thr.join();
        for (const Segment &seg : g.inflight) {
            hipEventSynchronize(seg.copied);
            hipEventDestroy(seg.copied);
        }
        for (hipEvent_t e : g.spare) hipEventDestroy(e);
        if (g.buf) hipHostFree(g.buf);
    }
    for (int k = 0; k < kStreams; ++k) {
        if (s->compute[k]) hipStreamSynchronize(s->compute[k]);
        for (hb_plan *pl : s->plan[k])
            if (pl) hb_plan_destroy(pl);
        if (s->h_meta[k]) hipHostFree(s->h_meta[k]);
        if (s->d_meta[k]) hipFree(s->d_meta[k]);
        if (s->compute[k]) hipStreamDestroy(s->compute[k]);
    }
    if (s->r_stream) hipStreamDestroy(s->r_stream);  // the launch ended above
    if (s->r_ev) hipEventDestroy(s->r_ev);
    for (void *h : {static_cast<void *>(s->r_items), static_cast<void *>(s->r_ctl), static_cast<void *>(s->r_done),
                    static_cast<void *>(s->r_off), static_cast<void *>(s->r_len), static_cast<void *>(s->r_slot),
                    static_cast<void *>(s->r_dig)})
        if (h) hipHostFree(h);
    if (s->r_dev) hipFree(s->r_dev);
    for (hipStream_t c : s->copy_in) {
        if (!c) continue;
        hipStreamSynchronize(c);
        hipStreamDestroy(c);
    }
    for (auto &q : s->unseen) q.clear();
    for (hipEvent_t e : s->ev_pool) hipEventDestroy(e);
    if (s->d_arena) hipFree(s->d_arena);
    delete s;
}

}  // extern "C"
