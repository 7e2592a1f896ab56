// Job state transitions of the gridding server (host only, no HIP types), so
// that they can be unit-tested on the CPU.
#pragma once

#include <cstddef>
#include <cstdint>

namespace mg {

// What the completion query of a running job's event reported.
enum class EventQuery { kDone, kNotReady, kError };

// Job states, numbered as mg_job_state.
enum : int { kJobQueued = 0, kJobRunning = 1, kJobDone = 2, kJobFailed = 3 };

struct JobAccount {
    int state = kJobQueued;
    int status = 0;            // mg_status of the job (0 = MG_OK)
    size_t footprint = 0;      // HBM bytes admitted for the job
};

struct ServerAccount {
    uint64_t bytes_in_use = 0;
    uint64_t completed = 0;
    uint64_t failed = 0;
};

// Applies one completion query to a running job.  Done: the job completes.
// Not ready: nothing changes.  Any other result (a device error reported for
// the job's work): the job fails with `device_error_status`.  A finished job
// releases its footprint and is counted once.  Returns true if the job left
// the running state.
inline bool settle_running_job(JobAccount &j, EventQuery q, ServerAccount &s,
                               int device_error_status) {
    if (j.state != kJobRunning || q == EventQuery::kNotReady) return false;
    if (q == EventQuery::kDone) {
        j.state = kJobDone;
        s.completed++;
    } else {
        j.state = kJobFailed;
        j.status = device_error_status;
        s.failed++;
    }
    s.bytes_in_use -= j.footprint;
    return true;
}

}  // namespace mg
