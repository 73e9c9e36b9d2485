// Host-only stand-in for the HIP calls of the serving loop; see hip/hip_runtime.h here.
#include "fake_hip.hpp"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <random>
#include <thread>
#include <unordered_set>

struct FakeEvent {
    uint64_t recorded = 0;   // generation of the latest record
    uint64_t completed = 0;  // latest generation whose record op has run
    long pending_waits = 0;  // queued stream waits on this event not yet satisfied
    bool alive = true;
};

namespace {

struct Op {
    enum Kind { Copy, Record, Wait, Fn } kind;
    void *dst = nullptr;
    const void *src = nullptr;
    size_t n = 0;
    FakeEvent *ev = nullptr;
    uint64_t gen = 0;
    std::function<void()> fn;
};

std::mutex g_mu;                // guards all state below and every stream's queue
std::condition_variable g_cv;   // any op finished
FakeHipReport g_rep;
long g_events_in_flight = 0;
// every event and stream ever created: kept (never freed, so late use is caught), and the
// sets themselves outlive static destruction, so the leak checker sees them reachable
std::unordered_set<FakeEvent *> &g_events = *new std::unordered_set<FakeEvent *>();

void violation(const std::string &what)
{
    g_rep.violations++;
    if (g_rep.first_violation.empty()) g_rep.first_violation = what;
}

}  // namespace

struct FakeStream {
    std::deque<Op> q;
    std::thread thr;
    bool stop = false;
    bool alive = true;
    std::mt19937 rng{12345};

    void run()
    {
        std::unique_lock<std::mutex> lk(g_mu);
        for (;;) {
            g_cv.wait(lk, [&] { return stop || !q.empty(); });
            if (q.empty()) return;
            Op &op = q.front();
            switch (op.kind) {
            case Op::Wait:
                g_cv.wait(lk, [&] { return op.ev->completed >= op.gen; });
                op.ev->pending_waits--;
                break;
            case Op::Copy: {
                const unsigned jitter = rng() % 4 == 0 ? rng() % 40 : 0;  // shuffle timings
                lk.unlock();
                if (jitter) std::this_thread::sleep_for(std::chrono::microseconds(jitter));
                std::memcpy(op.dst, op.src, op.n);
                lk.lock();
                break;
            }
            case Op::Fn: {
                auto fn = std::move(op.fn);
                const unsigned jitter = rng() % 4 == 0 ? rng() % 100 : 0;
                lk.unlock();
                if (jitter) std::this_thread::sleep_for(std::chrono::microseconds(jitter));
                fn();
                lk.lock();
                break;
            }
            case Op::Record:
                if (op.gen > op.ev->completed) {
                    if (op.ev->recorded == op.gen) g_events_in_flight--;  // its latest record is done
                    op.ev->completed = op.gen;
                }
                break;
            }
            q.pop_front();
            g_cv.notify_all();
        }
    }
};

namespace {

std::unordered_set<FakeStream *> &g_streams = *new std::unordered_set<FakeStream *>();

bool live_stream(hipStream_t s, const char *what)
{
    if (!s || !g_streams.count(s) || !s->alive) {
        violation(std::string(what) + ": unknown or destroyed stream");
        return false;
    }
    return true;
}

bool live_event(hipEvent_t e, const char *what)
{
    if (!e || !g_events.count(e) || !e->alive) {
        violation(std::string(what) + ": unknown or destroyed event");
        return false;
    }
    return true;
}

void push(hipStream_t s, Op op)
{
    s->q.push_back(std::move(op));
    g_rep.max_ops_in_flight = std::max<long>(g_rep.max_ops_in_flight, long(s->q.size()));
    g_cv.notify_all();
}

}  // namespace

hipError_t fake_hip_launch(hipStream_t stream, std::function<void()> fn)
{
    std::lock_guard<std::mutex> g(g_mu);
    if (!live_stream(stream, "launch")) return hipErrorInvalidResourceHandle;
    Op op{Op::Fn};
    op.fn = std::move(fn);
    push(stream, std::move(op));
    return hipSuccess;
}

FakeHipReport fake_hip_report()
{
    std::lock_guard<std::mutex> g(g_mu);
    return g_rep;
}

hipError_t hipSetDevice(int) { return hipSuccess; }

hipError_t hipMalloc(void **ptr, size_t size)
{
    *ptr = std::aligned_alloc(256, (size + 255) & ~size_t(255));
    return *ptr ? hipSuccess : hipErrorOutOfMemory;
}

hipError_t hipFree(void *ptr)
{
    std::free(ptr);
    return hipSuccess;
}

hipError_t hipHostMalloc(void **ptr, size_t size, unsigned int) { return hipMalloc(ptr, size); }
hipError_t hipHostFree(void *ptr) { return hipFree(ptr); }

hipError_t hipHostGetDevicePointer(void **dptr, void *hptr, unsigned int)
{
    *dptr = hptr;
    return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t *stream, unsigned int)
{
    auto *s = new FakeStream();
    {
        std::lock_guard<std::mutex> g(g_mu);
        g_streams.insert(s);
        s->rng.seed(unsigned(g_streams.size()) * 7919u);
    }
    s->thr = std::thread([s] { s->run(); });
    *stream = s;
    return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t stream)
{
    std::unique_lock<std::mutex> lk(g_mu);
    if (!live_stream(stream, "hipStreamSynchronize")) return hipErrorInvalidResourceHandle;
    g_cv.wait(lk, [&] { return stream->q.empty(); });
    return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t stream)
{
    {
        std::unique_lock<std::mutex> lk(g_mu);
        if (!live_stream(stream, "hipStreamDestroy")) return hipErrorInvalidResourceHandle;
        g_cv.wait(lk, [&] { return stream->q.empty(); });  // queued work still completes
        stream->alive = false;
        stream->stop = true;
        g_cv.notify_all();
    }
    stream->thr.join();  // the stream object itself is kept, so late use is caught
    return hipSuccess;
}

hipError_t hipStreamWaitEvent(hipStream_t stream, hipEvent_t event, unsigned int)
{
    std::lock_guard<std::mutex> g(g_mu);
    if (!live_stream(stream, "hipStreamWaitEvent") || !live_event(event, "hipStreamWaitEvent"))
        return hipErrorInvalidResourceHandle;
    if (event->recorded == 0) {  // a wait on an event never recorded does nothing
        g_rep.waits_unrecorded++;
        return hipSuccess;
    }
    Op op{Op::Wait};
    op.ev = event;
    op.gen = event->recorded;
    event->pending_waits++;
    push(stream, std::move(op));
    return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t *event, unsigned int)
{
    auto *e = new FakeEvent();
    std::lock_guard<std::mutex> g(g_mu);
    g_events.insert(e);
    g_rep.events_created++;
    *event = e;
    return hipSuccess;
}

hipError_t hipEventDestroy(hipEvent_t event)
{
    std::lock_guard<std::mutex> g(g_mu);
    if (!live_event(event, "hipEventDestroy")) return hipErrorInvalidResourceHandle;
    if (event->recorded > event->completed) violation("hipEventDestroy: the event's record has not completed");
    if (event->pending_waits > 0) violation("hipEventDestroy: a stream still waits on the event");
    event->alive = false;
    g_rep.events_destroyed++;
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t event, hipStream_t stream)
{
    std::lock_guard<std::mutex> g(g_mu);
    if (!live_stream(stream, "hipEventRecord") || !live_event(event, "hipEventRecord"))
        return hipErrorInvalidResourceHandle;
    if (event->recorded > event->completed) g_rep.rerecords_in_flight++;
    else g_events_in_flight++;
    g_rep.max_events_in_flight = std::max(g_rep.max_events_in_flight, g_events_in_flight);
    Op op{Op::Record};
    op.ev = event;
    op.gen = ++event->recorded;
    push(stream, std::move(op));
    return hipSuccess;
}

hipError_t hipEventQuery(hipEvent_t event)
{
    std::lock_guard<std::mutex> g(g_mu);
    if (!live_event(event, "hipEventQuery")) return hipErrorInvalidResourceHandle;
    return event->completed >= event->recorded ? hipSuccess : hipErrorNotReady;
}

hipError_t hipEventSynchronize(hipEvent_t event)
{
    std::unique_lock<std::mutex> lk(g_mu);
    if (!live_event(event, "hipEventSynchronize")) return hipErrorInvalidResourceHandle;
    const uint64_t want = event->recorded;
    g_cv.wait(lk, [&] { return event->completed >= want; });
    return hipSuccess;
}

hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind, hipStream_t stream)
{
    std::lock_guard<std::mutex> g(g_mu);
    if (!live_stream(stream, "hipMemcpyAsync")) return hipErrorInvalidResourceHandle;
    Op op{Op::Copy};
    op.dst = dst;
    op.src = src;
    op.n = n;
    push(stream, std::move(op));
    return hipSuccess;
}

hipError_t hipMemset(void *dst, int value, size_t n)
{
    std::memset(dst, value, n);
    return hipSuccess;
}

hipError_t hipDeviceGetAttribute(int *value, hipDeviceAttribute_t, int)
{
    *value = 8;  // "CUs" of the stand-in device
    return hipSuccess;
}

const char *hipGetErrorString(hipError_t e)
{
    switch (e) {
    case hipSuccess: return "hipSuccess";
    case hipErrorNotReady: return "hipErrorNotReady";
    case hipErrorOutOfMemory: return "hipErrorOutOfMemory";
    case hipErrorInvalidResourceHandle: return "hipErrorInvalidResourceHandle";
    default: return "hipErrorInvalidValue";
    }
}
