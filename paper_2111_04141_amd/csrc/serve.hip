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
    size_t footprint = 0;
    Clock::time_point t_submit, t_done;
    mg_job_state state = MG_JOB_QUEUED;
    mg_status status = MG_OK;
    hipEvent_t done_ev = nullptr;
};

}  // namespace
}  // namespace mg

struct mg_server {
    int device = 0;
    size_t budget = 0;
    int max_slots = 1;
    std::vector<hipStream_t> streams;
    size_t next_stream = 0;
    std::mutex mu;
    std::condition_variable cv_work;    // wakes the scheduler
    std::condition_variable cv_done;    // wakes waiters
    std::deque<uint64_t> pending;
    std::vector<uint64_t> running;
    std::unordered_map<uint64_t, std::unique_ptr<mg::Job>> jobs;
    uint64_t next_id = 1;
    mg_server_stats stats{};
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
    const size_t tiles8 = (size_t)((g->nu + 7) / 8) * (size_t)((g->nv + 7) / 8);
    const size_t nb = (size_t)np * tiles8;                      // buckets (tiles >= 8)
    const size_t caller = n * 3 * dtype_bytes(uvw_dtype) + n * g->npol * 8 +
                          (size_t)g->npol * g->nu * g->nv * 8;
    // the plan's table (no larger than the caller's) and its conjugate copy
    const size_t taps = (size_t)k->ntaps * dtype_bytes(k->tap_dtype) *
                        (k->kind == MG_KERNEL_WPROJ ? 4 : 1);
    // per record: sorted meta, permutation, sorted visibilities; per bucket:
    // count, start, cursor, first chunk, chunk, unit; per R-chunk (R >= 64):
    // chunk, unit
    const size_t scratch = n * (8 + 4 + 32) + nb * (4 * 4 + 16 + 8) +
                           (n / 64 + 1) * 24 + (1u << 20);
    return caller + taps + scratch;
}

void scheduler_loop(mg_server *s) {
    hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // completions
        bool finished = false;
        for (size_t i = 0; i < s->running.size();) {
            Job &j = *s->jobs[s->running[i]];
            if (hipEventQuery(j.done_ev) == hipSuccess) {
                j.t_done = Clock::now();
                j.state = MG_JOB_DONE;
                hipEventDestroy(j.done_ev);
                j.done_ev = nullptr;
                s->stats.bytes_in_use -= j.footprint;
                s->stats.completed++;
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
            if (s->stats.bytes_in_use + j.footprint > s->budget) break;
            s->pending.pop_front();
            s->stats.bytes_in_use += j.footprint;
            s->stats.bytes_peak = std::max(s->stats.bytes_peak, s->stats.bytes_in_use);
            s->stats.admitted++;
            j.state = MG_JOB_RUNNING;
            s->running.push_back(j.id);
            s->stats.max_running = std::max<int32_t>(s->stats.max_running, (int32_t)s->running.size());
            hipStream_t st = s->streams[s->next_stream++ % s->streams.size()];
            lk.unlock();
            mg_status rc = mg_grid(&j.g, &j.k, j.nrec, j.uvw, j.uvw_dtype, j.vis, j.grid, nullptr, st);
            hipEvent_t ev = nullptr;
            if (rc == MG_OK && (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
                                hipEventRecord(ev, st) != hipSuccess))
                rc = MG_EDEVICE;
            lk.lock();
            if (rc != MG_OK) {
                if (ev) hipEventDestroy(ev);
                j.status = rc;
                j.state = MG_JOB_FAILED;
                j.t_done = Clock::now();
                s->stats.bytes_in_use -= j.footprint;
                s->stats.failed++;
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
                           int32_t nstreams) {
    if (!srv) return set_error(MG_EINVAL, "null server output");
    *srv = nullptr;
    if (hbm_budget_bytes == 0) return set_error(MG_EINVAL, "zero budget");
    if (max_slots < 1 || max_slots > 1024) return set_error(MG_EINVAL, "max_slots must be in 1..1024");
    if (nstreams < 1 || nstreams > 64) return set_error(MG_EINVAL, "nstreams must be in 1..64");
    auto s = std::make_unique<mg_server>();
    if (hipGetDevice(&s->device) != hipSuccess) return set_error(MG_EDEVICE, "no device");
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    s->stats.budget = hbm_budget_bytes;
    for (int i = 0; i < nstreams; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t x : s->streams) hipStreamDestroy(x);
            return set_error(MG_EDEVICE, "stream creation failed");
        }
        s->streams.push_back(st);
    }
    mg_server *raw = s.get();
    raw->worker = std::thread(scheduler_loop, raw);
    *srv = s.release();
    return MG_OK;
}

mg_status mg_server_submit(mg_server *s, const mg_grid_desc *g, const mg_kernel_desc *k,
                           int64_t nrec, const void *uvw, mg_dtype uvw_dtype, const void *vis,
                           void *grid, uint64_t *job_id) {
    if (!s || !job_id) return set_error(MG_EINVAL, "null server or job id");
    if (!g || !k) return set_error(MG_EINVAL, "null descriptor");
    if (nrec > 0 && !vis) return set_error(MG_EINVAL, "null vis");
    if (!grid) return set_error(MG_EINVAL, "null grid");
    if (nrec < 0) return set_error(MG_EINVAL, "negative nrec");
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
    j->footprint = job_footprint(g, k, nrec, uvw_dtype);
    if (j->footprint > s->budget)
        return set_error(MG_ENOMEM, "job footprint exceeds the server's HBM budget");
    j->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) return set_error(MG_EBUSY, "server is shutting down");
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
    *state = j.state;
    if (latency_s)
        *latency_s = (j.state == MG_JOB_DONE || j.state == MG_JOB_FAILED)
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
    s->cv_done.wait(lk, [&] { return j.state == MG_JOB_DONE || j.state == MG_JOB_FAILED; });
    if (latency_s) *latency_s = std::chrono::duration<double>(j.t_done - j.t_submit).count();
    return j.state == MG_JOB_DONE ? MG_OK : j.status;
}

mg_status mg_server_get_stats(mg_server *s, mg_server_stats *out) {
    if (!s || !out) return set_error(MG_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
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
    for (hipStream_t st : s->streams) {
        hipStreamSynchronize(st);
        hipStreamDestroy(st);
    }
    delete s;
    return MG_OK;
}

}  // extern "C"
