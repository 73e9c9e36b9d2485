// Extra hooks of the host-only HIP stand-in (hip/hip_runtime.h beside this file).
#pragma once

#include <functional>
#include <string>

#include <hip/hip_runtime.h>

// Enqueue host work on a stand-in stream, run in stream order (a "kernel").
hipError_t fake_hip_launch(hipStream_t stream, std::function<void()> fn);

// Rule violations and counts seen so far; violations() == 0 means every rule was kept.
struct FakeHipReport {
    long violations = 0;           // destroyed while in flight, used after destroy, ...
    long rerecords_in_flight = 0;  // an event recorded again before its last record completed
    long waits_unrecorded = 0;     // waits on an event never recorded
    long max_ops_in_flight = 0;    // most ops queued on one stream at once
    long max_events_in_flight = 0; // most events recorded and not yet complete at once
    long events_created = 0, events_destroyed = 0;
    std::string first_violation;
};
FakeHipReport fake_hip_report();
