// Serving: continuous batching of gridding jobs (host scheduler).
//
// Jobs are queued by mg_server_submit and admitted in arrival order by a
// scheduler thread whenever a slot is free and the job's HBM footprint fits
// the budget beside the running jobs.  Each admitted job runs the one-shot
// gridding pipeline (index, bucket sort, chunk sort, gather, gridding
// kernels) on the next stream of a pool, so jobs that arrive while others
// run share the device.  Completion is observed through a per-job event;
// the job's footprint is then released and queued jobs can be admitted.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "serve_state.h"

using Clock = std::chrono::steady_clock;

namespace mg {
namespace {

struct Job {
    uint64_t id = 0;
    mg_grid_desc g{};
    mg_kernel_desc k{};
    std::vector<int32_t> plane_support;
    std::vector<int64_t> plane_offset;
    int64_t nrec = 0;
    const void *uvw = nullptr;
    mg_dtype uvw_dtype = MG_F32;
    const void *vis = nullptr;
    void *grid = nullptr;
    JobAccount acct;
    Clock::time_point t_submit, t_done;
    hipEvent_t ready_ev = nullptr;   // inputs ready (library event), may be null
    hipEvent_t done_ev = nullptr;
};

}  // namespace
}  // namespace mg

struct mg_server {
    int device = 0;
    size_t budget = 0;
    int max_slots = 1;
    std::vector<hipStream_t> streams;
    std::vector<void *> arenas;         // per stream: plan and scratch of its jobs
    std::vector<size_t> arena_bytes;
    hipStream_t gate = nullptr;        // orders submit-time event waits
    size_t next_stream = 0;
    std::mutex mu;
    std::condition_variable cv_work;    // wakes the scheduler
    std::condition_variable cv_done;    // wakes waiters
    std::deque<uint64_t> pending;
    std::vector<uint64_t> running;
    std::unordered_map<uint64_t, std::unique_ptr<mg::Job>> jobs;
    std::vector<hipEvent_t> free_events;   // reused job events
    uint64_t next_id = 1;
    mg_server_stats stats{};
    mg::ServerAccount acct;
    bool stopping = false;
    std::thread worker;
};

namespace mg {
namespace {

size_t dtype_bytes(mg_dtype d) { return d == MG_F64 ? 8 : d == MG_F32 ? 4 : 2; }

// Upper bound of the device memory one job holds: its caller buffers plus
// the scratch of the one-shot pipeline (plan arrays, temporaries, sorted
// visibilities, private tap table).
size_t job_footprint(const mg_grid_desc *g, const mg_kernel_desc *k, int64_t nrec,
                     mg_dtype uvw_dtype) {
    const size_t n = (size_t)nrec + kRecPad;
    const int np = k->kind == MG_KERNEL_WPROJ ? k->nplanes : 1;
    // W-stacking: the layers are stacked along v, one plane of buckets
    const size_t rows = (size_t)g->nv * (k->kind == MG_KERNEL_WSTACK ? (size_t)k->nplanes : 1u);
    const size_t tiles8 = (size_t)((g->nu + 7) / 8) * ((rows + 7) / 8);
    const size_t nb = (size_t)np * tiles8;                      // buckets (tiles >= 8)
    const size_t caller = n * 3 * dtype_bytes(uvw_dtype) + n * g->npol * 8 +
                          (size_t)g->npol * g->nu * rows * 8;
    // the plan's table (no larger than the caller's) and its conjugate copy
    const size_t taps = (size_t)k->ntaps * dtype_bytes(k->tap_dtype) *
                        (k->kind == MG_KERNEL_WPROJ ? 4 : 1);
    // per record: sorted meta, permutation, sorted visibilities; per bucket:
    // count, start, cursor, first chunk, chunk, unit, unit word; per
    // R-chunk (R >= 64): chunk, unit, unit word
    const size_t scratch = n * (8 + 4 + 32) + nb * (4 * 4 + 16 + 8 + 4) +
                           (n / 64 + 1) * 28 + (1u << 20);
    return caller + taps + scratch;
}

hipEvent_t take_event(mg_server *s) {
    if (!s->free_events.empty()) {
        hipEvent_t e = s->free_events.back();
        s->free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

void give_event(mg_server *s, hipEvent_t &e) {
    if (e) s->free_events.push_back(e);
    e = nullptr;
}

EventQuery query(hipEvent_t e) {
    const hipError_t r = hipEventQuery(e);
    if (r == hipSuccess) return EventQuery::kDone;
    if (r == hipErrorNotReady) return EventQuery::kNotReady;
    return EventQuery::kError;
}

void scheduler_loop(mg_server *s) {
    hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // completions (a device error reported for a job's work fails the job)
        bool finished = false;
        for (size_t i = 0; i < s->running.size();) {
            Job &j = *s->jobs[s->running[i]];
            if (settle_running_job(j.acct, query(j.done_ev), s->acct, MG_EDEVICE)) {
                j.t_done = Clock::now();
                give_event(s, j.done_ev);
                give_event(s, j.ready_ev);
                s->running.erase(s->running.begin() + i);
                finished = true;
            } else {
                ++i;
            }
        }
        if (finished) s->cv_done.notify_all();
        // admissions, in arrival order
        while (!s->pending.empty() && (int)s->running.size() < s->max_slots) {
            Job &j = *s->jobs[s->pending.front()];
            if (s->acct.bytes_in_use + j.acct.footprint > s->budget) break;
            s->pending.pop_front();
            s->acct.bytes_in_use += j.acct.footprint;
            s->stats.bytes_peak = std::max<uint64_t>(s->stats.bytes_peak, s->acct.bytes_in_use);
            s->stats.admitted++;
            j.acct.state = kJobRunning;
            s->running.push_back(j.id);
            s->stats.max_running = std::max<int32_t>(s->stats.max_running, (int32_t)s->running.size());
            const size_t si = s->next_stream++ % s->streams.size();
            hipStream_t st = s->streams[si];
            hipEvent_t ev = take_event(s);
            hipEvent_t ready = j.ready_ev;
            lk.unlock();
            mg_status rc = MG_OK;
            if (ready && hipStreamWaitEvent(st, ready, 0) != hipSuccess) rc = MG_EDEVICE;
            if (rc == MG_OK)
                rc = grid_in_arena(&j.g, &j.k, j.nrec, j.uvw, j.uvw_dtype, j.vis, j.grid,
                                   &s->arenas[si], &s->arena_bytes[si], st);
            if (rc == MG_OK && (!ev || hipEventRecord(ev, st) != hipSuccess)) rc = MG_EDEVICE;
            lk.lock();
            if (rc != MG_OK) {
                give_event(s, ev);
                give_event(s, j.ready_ev);
                j.acct.status = rc;
                j.acct.state = kJobFailed;
                j.t_done = Clock::now();
                s->acct.bytes_in_use -= j.acct.footprint;
                s->acct.failed++;
                s->running.erase(std::find(s->running.begin(), s->running.end(), j.id));
                s->cv_done.notify_all();
            } else {
                j.done_ev = ev;
            }
        }
        s->stats.running = (int32_t)s->running.size();
        s->stats.queued = (int32_t)s->pending.size();
        if (s->stopping && s->pending.empty() && s->running.empty()) break;
        if (s->running.empty())
            s->cv_work.wait(lk);
        else
            s->cv_work.wait_for(lk, std::chrono::microseconds(20));
    }
}

}  // namespace
}  // namespace mg

using namespace mg;

extern "C" {

mg_status mg_server_create(mg_server **srv, size_t hbm_budget_bytes, int32_t max_slots,
                           int32_t nstreams, int32_t device) {
    if (!srv) return set_error(MG_EINVAL, "null server output");
    *srv = nullptr;
    if (hbm_budget_bytes == 0) return set_error(MG_EINVAL, "zero budget");
    if (max_slots < 1 || max_slots > 1024) return set_error(MG_EINVAL, "max_slots must be in 1..1024");
    if (nstreams < 1 || nstreams > 64) return set_error(MG_EINVAL, "nstreams must be in 1..64");
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return set_error(MG_EDEVICE, "no device");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < -1 || device >= ndev)
        return set_error(MG_EINVAL, "device out of range");
    auto s = std::make_unique<mg_server>();
    s->device = device < 0 ? prev : device;
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    s->stats.budget = hbm_budget_bytes;
    if (hipSetDevice(s->device) != hipSuccess) return set_error(MG_EDEVICE, "cannot select device");
    bool ok = true;
    for (int i = 0; i < nstreams + 1 && ok; ++i) {
        hipStream_t st;
        ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        if (ok && i < nstreams) {
            s->streams.push_back(st);
            s->arenas.push_back(nullptr);
            s->arena_bytes.push_back(0);
        }
        if (ok && i == nstreams) s->gate = st;
    }
    hipSetDevice(prev);
    if (!ok) {
        for (hipStream_t x : s->streams) hipStreamDestroy(x);
        return set_error(MG_EDEVICE, "stream creation failed");
    }
    mg_server *raw = s.get();
    raw->worker = std::thread(scheduler_loop, raw);
    *srv = s.release();
    return MG_OK;
}

mg_status mg_server_submit(mg_server *s, const mg_grid_desc *g, const mg_kernel_desc *k,
                           int64_t nrec, const void *uvw, mg_dtype uvw_dtype, const void *vis,
                           void *grid, hipEvent_t inputs_ready, uint64_t *job_id) {
    if (!s || !job_id) return set_error(MG_EINVAL, "null server or job id");
    if (!g || !k) return set_error(MG_EINVAL, "null descriptor");
    if (nrec > 0 && !vis) return set_error(MG_EINVAL, "null vis");
    if (!grid) return set_error(MG_EINVAL, "null grid");
    if (nrec < 0) return set_error(MG_EINVAL, "negative nrec");
    if (k->kind == MG_KERNEL_WSTACK &&
        (k->nplanes < 1 || k->nplanes > 128 || (int64_t)k->nplanes * g->nv > 65535))
        return set_error(MG_EINVAL, "W-stacking layers must be in [1, 128] with layers x nv <= 65535");
    if (k->kind == MG_KERNEL_WPROJ && (k->nplanes < 1 || k->nplanes > kMaxPlanes ||
                                       !k->plane_support || !k->plane_offset))
        return set_error(MG_EINVAL, "bad W-projection planes");
    auto j = std::make_unique<Job>();
    j->g = *g;
    j->k = *k;
    if (k->kind == MG_KERNEL_WPROJ) {
        j->plane_support.assign(k->plane_support, k->plane_support + k->nplanes);
        j->plane_offset.assign(k->plane_offset, k->plane_offset + k->nplanes);
        j->k.plane_support = j->plane_support.data();
        j->k.plane_offset = j->plane_offset.data();
    }
    j->nrec = nrec;
    j->uvw = uvw;
    j->uvw_dtype = uvw_dtype;
    j->vis = vis;
    j->grid = grid;
    j->acct.footprint = job_footprint(g, k, nrec, uvw_dtype);
    if (j->acct.footprint > s->budget)
        return set_error(MG_ENOMEM, "job footprint exceeds the server's HBM budget");
    j->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) return set_error(MG_EBUSY, "server is shutting down");
        if (inputs_ready) {
            // a library event that completes with the caller's: the caller
            // may re-record or destroy its event once submit returns
            hipEvent_t ev = take_event(s);
            if (!ev || hipStreamWaitEvent(s->gate, inputs_ready, 0) != hipSuccess ||
                hipEventRecord(ev, s->gate) != hipSuccess) {
                give_event(s, ev);
                return set_error(MG_EDEVICE, "input event wait failed");
            }
            j->ready_ev = ev;
        }
        j->id = s->next_id++;
        *job_id = j->id;
        s->pending.push_back(j->id);
        s->jobs.emplace(j->id, std::move(j));
        s->stats.submitted++;
    }
    s->cv_work.notify_one();
    return MG_OK;
}

mg_status mg_server_poll(mg_server *s, uint64_t job_id, mg_job_state *state, double *latency_s) {
    if (!s || !state) return set_error(MG_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return set_error(MG_EINVAL, "unknown job id");
    const Job &j = *it->second;
    *state = (mg_job_state)j.acct.state;
    if (latency_s)
        *latency_s = (j.acct.state == kJobDone || j.acct.state == kJobFailed)
                         ? std::chrono::duration<double>(j.t_done - j.t_submit).count()
                         : -1.0;
    return MG_OK;
}

mg_status mg_server_wait(mg_server *s, uint64_t job_id, double *latency_s) {
    if (!s) return set_error(MG_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return set_error(MG_EINVAL, "unknown job id");
    Job &j = *it->second;
    s->cv_done.wait(lk, [&] { return j.acct.state == kJobDone || j.acct.state == kJobFailed; });
    if (latency_s) *latency_s = std::chrono::duration<double>(j.t_done - j.t_submit).count();
    const mg_status st = j.acct.state == kJobDone ? MG_OK : (mg_status)j.acct.status;
    s->jobs.erase(it);
    if (st != MG_OK) return set_error(st, "job failed");
    return MG_OK;
}

mg_status mg_server_get_stats(mg_server *s, mg_server_stats *out) {
    if (!s || !out) return set_error(MG_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->bytes_in_use = s->acct.bytes_in_use;
    out->completed = s->acct.completed;
    out->failed = s->acct.failed;
    return MG_OK;
}

mg_status mg_server_destroy(mg_server *s) {
    if (!s) return MG_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_one();
    if (s->worker.joinable()) s->worker.join();
    for (size_t i = 0; i < s->streams.size(); ++i) {
        if (s->arenas[i]) scratch_free(s->arenas[i], s->streams[i]);
        hipStreamSynchronize(s->streams[i]);
        hipStreamDestroy(s->streams[i]);
    }
    if (s->gate) {
        hipStreamSynchronize(s->gate);
        hipStreamDestroy(s->gate);
    }
    for (auto &kv : s->jobs) {
        if (kv.second->done_ev) hipEventDestroy(kv.second->done_ev);
        if (kv.second->ready_ev) hipEventDestroy(kv.second->ready_ev);
    }
    for (hipEvent_t e : s->free_events) hipEventDestroy(e);
    delete s;
    return MG_OK;
}

}  // extern "C"
