// CPU unit test of the gridding server's job state transitions
// (paper_2111_04141_amd/csrc/serve_state.h); built and run by
// tests/test_serve_state.py.  Exit status 0 on success.
#include <cstdio>

#include "serve_state.h"

using namespace mg;

static int fails = 0;
#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            std::printf("FAILED line %d: %s\n", __LINE__, #c);     \
            ++fails;                                               \
        }                                                          \
    } while (0)

int main() {
    const int kDeviceError = -3;
    ServerAccount s;
    s.bytes_in_use = 300;
    // a running job whose event is not ready stays running
    JobAccount a;
    a.state = kJobRunning;
    a.footprint = 100;
    CHECK(!settle_running_job(a, EventQuery::kNotReady, s, kDeviceError));
    CHECK(a.state == kJobRunning && s.bytes_in_use == 300 && s.completed == 0);
    // completion releases the footprint once
    CHECK(settle_running_job(a, EventQuery::kDone, s, kDeviceError));
    CHECK(a.state == kJobDone && a.status == 0 && s.bytes_in_use == 200 && s.completed == 1);
    CHECK(!settle_running_job(a, EventQuery::kDone, s, kDeviceError));
    CHECK(s.bytes_in_use == 200 && s.completed == 1);
    // a device error fails the job (it must not stay running forever)
    JobAccount b;
    b.state = kJobRunning;
    b.footprint = 150;
    CHECK(settle_running_job(b, EventQuery::kError, s, kDeviceError));
    CHECK(b.state == kJobFailed && b.status == kDeviceError);
    CHECK(s.bytes_in_use == 50 && s.failed == 1 && s.completed == 1);
    CHECK(!settle_running_job(b, EventQuery::kError, s, kDeviceError));
    CHECK(s.failed == 1 && s.bytes_in_use == 50);
    // queued jobs are not touched by completion queries
    JobAccount c;
    c.footprint = 50;
    CHECK(!settle_running_job(c, EventQuery::kDone, s, kDeviceError));
    CHECK(c.state == kJobQueued && s.bytes_in_use == 50);
    if (fails == 0) std::printf("serve_state ok\n");
    return fails == 0 ? 0 : 1;
}
