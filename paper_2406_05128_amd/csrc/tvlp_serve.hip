// Serving runtime: continuous batching of filter jobs of different lengths.
//
// A server owns an HBM arena (sized by the caller's budget) holding each
// admitted job's excitation, coefficients and output, plus max_slots float64
// filter states.  A scheduler thread:
//   * admits queued jobs in arrival order while a slot and arena space are
//     free, uploading their inputs on an upload stream;
//   * every iteration, advances each running job by one slice of at most
//     `slice` samples from its device-resident state with one forward launch
//     over all slots (lp_forward_segments; idle slots have length 0);
//   * downloads finished outputs on a download stream and frees their space.
// Uploads and downloads overlap the compute stream.  A job's slice and chunk
// boundaries depend only on its own sample positions, and its state is
// carried in float64, so its result is bit-identical whether it runs alone or
// among other jobs.
#include "tvlp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

using Clock = std::chrono::steady_clock;

constexpr int64_t kAlign = 64;  // arena allocation granule, samples

// First-fit allocator over [0, capacity) in samples, coalescing on free.
class Arena {
  public:
    explicit Arena(int64_t capacity) { free_[0] = capacity; }
    bool alloc(int64_t n, int64_t &off) {
        n = (n + kAlign - 1) / kAlign * kAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                off = it->first;
                const int64_t rest = it->second - n;
                free_.erase(it);
                if (rest > 0) free_[off + n] = rest;
                return true;
            }
        }
        return false;
    }
    void release(int64_t off, int64_t n) {
        n = (n + kAlign - 1) / kAlign * kAlign;
        auto it = free_.emplace(off, n).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<int64_t, int64_t> free_;
};

enum class JobState { Queued, Uploading, Running, Downloading, Done, Failed };

struct Job {
    uint64_t ticket = 0;
    int64_t T = 0;
    const float *e_host = nullptr;
    const float *a_host = nullptr;
    float *s_host = nullptr;
    JobState state = JobState::Queued;
    int slot = -1;
    int64_t off = 0;  // arena offset in samples
    int64_t pos = 0;  // samples already filtered
    hipEvent_t ev_up = nullptr, ev_down = nullptr;
    // submitted, admitted (upload issued), first slice launched, last slice
    // finished on the device, output downloaded
    Clock::time_point t_submit, t_admit, t_first, t_computed, t_done;
    int status = LP_OK;
};

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

namespace tvlp_host {
int set_error(int code, const char *msg);
}

namespace {
int serve_fail(int code, const char *msg) { return tvlp_host::set_error(code, msg); }
}  // namespace

struct lp_server {
    int device = 0;
    int M = 0;
    int max_slots = 0;
    int64_t slice = 0;
    lp_plan *plan = nullptr;
    void *arena_mem = nullptr;
    float *e_arena = nullptr, *a_arena = nullptr, *s_arena = nullptr;
    int64_t arena_samples = 0;
    double *states = nullptr;
    int64_t *d_table = nullptr;  // [2][max_slots]: starts then lens
    int64_t *h_table = nullptr;  // pinned host copy
    hipStream_t s_up = nullptr, s_comp = nullptr, s_down = nullptr;
    Arena *arena = nullptr;

    std::thread thread;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    std::deque<Job *> queue;
    std::unordered_map<uint64_t, Job *> jobs;
    std::vector<Job *> slots;
    uint64_t next_ticket = 1;
    // statistics
    std::atomic<int64_t> iterations{0}, samples_done{0}, jobs_done{0};
    int fatal = LP_OK;

    void run();
    bool step_locked_free(std::unique_lock<std::mutex> &lk);
};

void lp_server::run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        // 1. admission in arrival order
        while (!queue.empty()) {
            Job *j = queue.front();
            auto it = std::find(slots.begin(), slots.end(), nullptr);
            if (it == slots.end()) break;
            int64_t off = 0;
            if (!arena->alloc(j->T, off)) break;
            queue.pop_front();
            j->slot = (int)(it - slots.begin());
            *it = j;
            j->off = off;
            j->state = JobState::Uploading;
            j->t_admit = Clock::now();
            hipError_t e1 = hipMemcpyAsync(e_arena + off, j->e_host, (size_t)j->T * sizeof(float),
                                           hipMemcpyHostToDevice, s_up);
            hipError_t e2 = hipMemcpyAsync(a_arena + off * M, j->a_host, (size_t)j->T * M * sizeof(float),
                                           hipMemcpyHostToDevice, s_up);
            hipError_t e3 = hipMemsetAsync(states + (size_t)j->slot * M, 0, (size_t)M * sizeof(double), s_up);
            hipError_t e4 = hipEventRecord(j->ev_up, s_up);
            if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess) {
                j->status = LP_EDEVICE;
                j->state = JobState::Failed;
                arena->release(j->off, j->T);
                *it = nullptr;
                cv.notify_all();
            }
        }
        // 2. uploads that have landed become runnable
        for (Job *j : slots)
            if (j && j->state == JobState::Uploading && hipEventQuery(j->ev_up) == hipSuccess)
                j->state = JobState::Running;
        // 3. one slice for every running job
        bool any = false;
        int64_t total = 0;
        for (int s = 0; s < max_slots; ++s) {
            Job *j = slots[s];
            int64_t start = 0, len = 0;
            if (j && j->state == JobState::Running) {
                len = std::min(slice, j->T - j->pos);
                start = j->off + j->pos;
                if (j->pos == 0) j->t_first = Clock::now();
                any = true;
            }
            h_table[s] = start;
            h_table[max_slots + s] = len;
            total += len;
        }
        if (any) {
            lk.unlock();
            int rc = LP_OK;
            if (hipMemcpyAsync(d_table, h_table, 2 * (size_t)max_slots * sizeof(int64_t), hipMemcpyHostToDevice,
                               s_comp) != hipSuccess)
                rc = LP_EDEVICE;
            if (rc == LP_OK)
                rc = lp_forward_segments(plan, max_slots, d_table, d_table + max_slots, arena_samples, total,
                                         e_arena, a_arena, states, s_arena, states, s_comp);
            // the next slice table overwrites h_table: finish this iteration first
            if (rc == LP_OK && hipStreamSynchronize(s_comp) != hipSuccess) rc = LP_EDEVICE;
            lk.lock();
            iterations++;
            for (int s = 0; s < max_slots; ++s) {
                Job *j = slots[s];
                if (!j || j->state != JobState::Running) continue;
                const int64_t len = h_table[max_slots + s];
                if (len <= 0) continue;
                if (rc != LP_OK) {
                    j->status = rc;
                    j->state = JobState::Failed;
                    arena->release(j->off, j->T);
                    slots[s] = nullptr;
                    continue;
                }
                j->pos += len;
                samples_done += len;
                if (j->pos >= j->T) {
                    // output complete: download, then release the arena space
                    j->t_computed = Clock::now();
                    j->state = JobState::Downloading;
                    slots[s] = nullptr;
                    if (hipMemcpyAsync(j->s_host, s_arena + j->off, (size_t)j->T * sizeof(float),
                                       hipMemcpyDeviceToHost, s_down) != hipSuccess ||
                        hipEventRecord(j->ev_down, s_down) != hipSuccess) {
                        j->status = LP_EDEVICE;
                        j->state = JobState::Failed;
                        arena->release(j->off, j->T);
                    }
                }
            }
            if (rc != LP_OK) fatal = rc;
            cv.notify_all();
        }
        // 4. downloads that have landed complete their jobs
        for (auto &kv : jobs) {
            Job *j = kv.second;
            if (j->state == JobState::Downloading && hipEventQuery(j->ev_down) == hipSuccess) {
                j->state = JobState::Done;
                j->t_done = Clock::now();
                arena->release(j->off, j->T);
                jobs_done++;
                cv.notify_all();
            }
        }
        // 5. idle handling
        bool busy = any;
        bool pending_io = false;
        for (auto &kv : jobs) {
            const JobState st = kv.second->state;
            if (st == JobState::Uploading || st == JobState::Downloading || st == JobState::Running) pending_io = true;
        }
        if (stop && queue.empty() && !pending_io) break;
        if (!busy) {
            if (pending_io) {
                cv.wait_for(lk, std::chrono::microseconds(20));
            } else {
                cv.wait_for(lk, std::chrono::milliseconds(2), [&] { return stop || !queue.empty(); });
            }
        }
    }
}

extern "C" {

int lp_serve_create(lp_server **out, int device, int M, size_t hbm_budget_bytes, int max_slots, int64_t slice_len,
                    int flags) {
    (void)flags;
    if (!out) return serve_fail(LP_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_slots < 1 || max_slots > 4096) return serve_fail(LP_EINVAL, "max_slots must be in [1, 4096]");
    lp_plan *plan = nullptr;
    int rc = lp_plan_create(&plan, device, M, 0);
    if (rc != LP_OK) return serve_fail(rc, lp_last_error());
    const int L = lp_plan_get_chunk(plan);
    if (slice_len <= 0) slice_len = 48 * L;
    slice_len = (slice_len + L - 1) / L * L;  // slices end on chunk boundaries of the job
    const size_t per_sample = (size_t)(M + 2) * sizeof(float);
    const int64_t samples = (int64_t)(hbm_budget_bytes / per_sample) / kAlign * kAlign;
    if (samples < kAlign) {
        lp_plan_destroy(plan);
        return serve_fail(LP_EINVAL, "HBM budget too small for any job");
    }
    lp_server *srv = new (std::nothrow) lp_server();
    if (!srv) {
        lp_plan_destroy(plan);
        return serve_fail(LP_ENOMEM, "out of host memory");
    }
    srv->device = device;
    srv->M = M;
    srv->max_slots = max_slots;
    srv->slice = slice_len;
    srv->plan = plan;
    srv->arena_samples = samples;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(device);
    bool ok = hipMalloc(&srv->arena_mem, (size_t)samples * per_sample) == hipSuccess &&
              hipMalloc(&srv->states, (size_t)max_slots * M * sizeof(double)) == hipSuccess &&
              hipMalloc(&srv->d_table, 2 * (size_t)max_slots * sizeof(int64_t)) == hipSuccess &&
              hipHostMalloc(&srv->h_table, 2 * (size_t)max_slots * sizeof(int64_t), hipHostMallocDefault) ==
                  hipSuccess &&
              hipStreamCreate(&srv->s_up) == hipSuccess && hipStreamCreate(&srv->s_comp) == hipSuccess &&
              hipStreamCreate(&srv->s_down) == hipSuccess;
    // workspace for the largest batch an iteration can launch, before any capture-free steady state
    if (ok) ok = lp_plan_reserve(plan, max_slots, slice_len) == LP_OK;
    if (ok) ok = hipMemset(srv->states, 0, (size_t)max_slots * M * sizeof(double)) == hipSuccess;
    (void)hipSetDevice(prev);
    if (!ok) {
        lp_serve_destroy(srv);
        return serve_fail(LP_ENOMEM, "device allocation for the server failed");
    }
    srv->e_arena = (float *)srv->arena_mem;
    srv->s_arena = srv->e_arena + samples;
    srv->a_arena = srv->s_arena + samples;
    srv->arena = new Arena(samples);
    srv->slots.assign(max_slots, nullptr);
    srv->thread = std::thread([srv] { srv->run(); });
    *out = srv;
    return LP_OK;
}

int lp_serve_submit(lp_server *srv, int64_t T, const float *e_host, const float *a_host, float *s_host_out,
                    uint64_t *ticket) {
    if (!srv || !ticket) return serve_fail(LP_EINVAL, "server or ticket is NULL");
    if (T < 1 || !e_host || !a_host || !s_host_out) return serve_fail(LP_EINVAL, "T >= 1 and host buffers required");
    if (T > srv->arena_samples) return serve_fail(LP_EBUDGET, "job larger than the whole HBM budget");
    Job *j = new (std::nothrow) Job();
    if (!j) return serve_fail(LP_ENOMEM, "out of host memory");
    j->T = T;
    j->e_host = e_host;
    j->a_host = a_host;
    j->s_host = s_host_out;
    j->t_submit = Clock::now();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(srv->device);
    const bool ok = hipEventCreateWithFlags(&j->ev_up, hipEventDisableTiming) == hipSuccess &&
                    hipEventCreateWithFlags(&j->ev_down, hipEventDisableTiming) == hipSuccess;
    (void)hipSetDevice(prev);
    if (!ok) {
        delete j;
        return serve_fail(LP_EDEVICE, "event creation failed");
    }
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        j->ticket = srv->next_ticket++;
        srv->jobs[j->ticket] = j;
        srv->queue.push_back(j);
        *ticket = j->ticket;
    }
    srv->cv.notify_all();
    return LP_OK;
}

}  // extern "C"

namespace {
int poll_impl(lp_server *srv, uint64_t ticket, double *latency_ms_out, double *device_ms_out) {
    if (!srv) return serve_fail(LP_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(ticket);
    if (it == srv->jobs.end()) return serve_fail(LP_ENOTFOUND, "unknown ticket");
    Job *j = it->second;
    if (j->state == JobState::Done || j->state == JobState::Failed) {
        const int st = j->status;
        if (latency_ms_out) *latency_ms_out = ms_between(j->t_submit, j->t_done);
        if (device_ms_out) *device_ms_out = st == LP_OK ? ms_between(j->t_first, j->t_computed) : 0.0;
        (void)hipEventDestroy(j->ev_up);
        (void)hipEventDestroy(j->ev_down);
        srv->jobs.erase(it);
        delete j;
        return st == LP_OK ? LP_OK : serve_fail(st, "job failed on the device");
    }
    return LP_PENDING;
}
}  // namespace

extern "C" {

int lp_serve_poll(lp_server *srv, uint64_t ticket, double *latency_ms_out) {
    return poll_impl(srv, ticket, latency_ms_out, nullptr);
}

int lp_serve_wait(lp_server *srv, uint64_t ticket, double timeout_s, double *latency_ms_out, double *device_ms_out) {
    if (!srv) return serve_fail(LP_EINVAL, "server is NULL");
    const Clock::time_point deadline =
        Clock::now() + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(timeout_s));
    for (;;) {
        const int rc = poll_impl(srv, ticket, latency_ms_out, device_ms_out);
        if (rc != LP_PENDING) return rc;
        std::unique_lock<std::mutex> lk(srv->mu);
        if (srv->cv.wait_until(lk, std::min(deadline, Clock::now() + std::chrono::milliseconds(1))) ==
                std::cv_status::timeout &&
            Clock::now() >= deadline)
            return LP_PENDING;
    }
}

int lp_serve_stats(lp_server *srv, int64_t *iterations, int64_t *samples, int64_t *jobs_done, int64_t *queued,
                   int64_t *active) {
    if (!srv) return serve_fail(LP_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (iterations) *iterations = srv->iterations;
    if (samples) *samples = srv->samples_done;
    if (jobs_done) *jobs_done = srv->jobs_done;
    if (queued) *queued = (int64_t)srv->queue.size();
    if (active) *active = (int64_t)std::count_if(srv->slots.begin(), srv->slots.end(), [](Job *j) { return j; });
    return LP_OK;
}

int lp_serve_destroy(lp_server *srv) {
    if (!srv) return LP_OK;
    if (srv->thread.joinable()) {
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->stop = true;
        }
        srv->cv.notify_all();
        srv->thread.join();
    }
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(srv->device);
    for (auto &kv : srv->jobs) {
        (void)hipEventDestroy(kv.second->ev_up);
        (void)hipEventDestroy(kv.second->ev_down);
        delete kv.second;
    }
    if (srv->s_up) (void)hipStreamDestroy(srv->s_up);
    if (srv->s_comp) (void)hipStreamDestroy(srv->s_comp);
    if (srv->s_down) (void)hipStreamDestroy(srv->s_down);
    if (srv->h_table) (void)hipHostFree(srv->h_table);
    if (srv->d_table) (void)hipFree(srv->d_table);
    if (srv->states) (void)hipFree(srv->states);
    if (srv->arena_mem) (void)hipFree(srv->arena_mem);
    (void)hipSetDevice(prev);
    if (srv->plan) lp_plan_destroy(srv->plan);
    delete srv->arena;
    delete srv;
    return LP_OK;
}

}  // extern "C"
