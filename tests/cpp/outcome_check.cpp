// Host check of how a serving request's failure reaches its caller: the failure is recorded
// on a worker thread (as a staging thread or the serving loop does), and the thread that
// waits for the request receives the status and its explanation in its own per-thread
// error slot; other threads' slots are untouched, and the first failure wins.
#include <condition_variable>
#include <cstdio>
#include <mutex>
#include <string>
#include <thread>

#include "../../paper_2407_09333_amd/csrc/hb_outcome.hpp"

namespace {

thread_local std::string t_error;  // stands for the library's per-thread last error
thread_local int t_status = 0;

void set_error(int st, const std::string &why)
{
    t_status = st;
    t_error = why;
}

struct Request {
    std::mutex mu;
    std::condition_variable cv;
    bool done = false;
    hb::Outcome res;
};

int fail(const char *what)
{
    std::printf("FAIL: %s\n", what);
    return 1;
}

}  // namespace

int main()
{
    // a worker fails the request; the waiter receives the text
    Request r;
    std::thread worker([&] {
        set_error(-3, "worker's own slot");
        std::lock_guard<std::mutex> g(r.mu);
        r.res.fail(-3, "hb_server: staging copy: out of memory");
        r.res.fail(-1, "a later consequence");  // ignored: the first failure wins
        r.done = true;
        r.cv.notify_all();
    });
    int status = 0;
    {
        std::unique_lock<std::mutex> g(r.mu);
        r.cv.wait(g, [&] { return r.done; });
        status = r.res.deliver(set_error);
    }
    worker.join();
    if (status != -3 || t_status != -3) return fail("status");
    if (t_error != "hb_server: staging copy: out of memory") return fail("text");

    // a third thread asking nothing keeps its own slot
    std::string other;
    std::thread bystander([&] { other = t_error; });
    bystander.join();
    if (!other.empty()) return fail("per-thread slot leaked");

    // a successful request delivers nothing and leaves the slot alone
    hb::Outcome ok;
    set_error(-5, "earlier unrelated error");
    if (ok.deliver(set_error) != 0 || t_error != "earlier unrelated error") return fail("ok outcome");

    // success recorded as a "failure" is ignored; an empty explanation gets a default
    hb::Outcome o;
    o.fail(0, "not a failure");
    if (o.status != 0) return fail("status 0 is not a failure");
    o.fail(-6, "");
    if (o.status != -6 || o.text.empty()) return fail("default text");

    std::printf("outcome ok\n");
    return 0;
}
