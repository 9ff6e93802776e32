// Ensemble serving: a continuous-batching loop over independent Richards
// simulations.  Requests wait in a FIFO queue and are admitted when a worker
// is free and their device-memory plan (rich_query_bytes) fits what the
// budget has left; every admitted simulation stays resident on the GPU for
// all of its steps, driven by its own worker thread on its own HIP stream,
// so the kernels of concurrent simulations overlap on the device.  With fused
// batching the preconditioned products of the simulations' GMRES solves go
// through a batcher, which issues them as batched launches over all posted
// simulations (the batcher itself lives with the solver).  Simulations share
// a batcher only when they have the same grid and precision: the blocks of a
// batched launch finish together, so a batch is only as fast as its largest
// member, while simulations of different classes keep overlapping on separate
// batcher streams.  Every block of a batched launch runs the lone kernel's
// code on its own simulation's data and all reductions are deterministic, so
// a simulation's result does not depend on what else is running.
#include <array>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "common.hpp"

namespace {

double wall_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    int64_t id = 0;
    rich_problem_t prob;
    rich_solver_opts_t opts;
    std::vector<double> ks, p;
    int nsteps = 0;
    size_t bytes = 0;
    int state = RICH_REQ_QUEUED;
    rich_status result = RICH_OK;
    std::vector<rich_step_stats_t> stats;
    std::vector<double> step_ms;
    double t_submit = 0, t_start = 0, t_end = 0;
    hipEvent_t after = nullptr;  // the server's stream at submission (null: no ordering)
};

}  // namespace

struct rich_server {
    size_t budget = 0, in_use = 0;
    int device = 0;
    hipStream_t order = nullptr;      // caller's stream each request is ordered after (may be null)
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::shared_ptr<Request>> queue;
    std::map<int64_t, std::shared_ptr<Request>> all;
    std::vector<std::thread> workers;
    int64_t next_id = 1;
    int running = 0;
    bool stop = false;
    int fused = 0;                    // fused batching of the preconditioned products: 0 off, 1 fused
                                      // launches, 2 persistent fused launches on a work queue
    // one batcher per class of (grid, precision), created with its first admission
    std::map<std::array<int, 4>, rich_batcher *> batchers;
};

namespace {

std::array<int, 4> batch_class(const Request &R) {
    return {R.prob.nx, R.prob.ny, R.prob.nz, R.opts.precision};
}

// Run one admitted request to completion on the worker's stream.
void run_request(rich_server *S, hipStream_t stream, Request &R, rich_batcher *batcher) {
    int64_t N = (int64_t)R.prob.nx * R.prob.ny * R.prob.nz;
    double *dks = nullptr, *dp = nullptr;
    rich_handle_t h = nullptr;
    rich_status st = RICH_OK;
    if (hipMalloc(&dks, N * sizeof(double)) != hipSuccess || hipMalloc(&dp, N * sizeof(double)) != hipSuccess)
        st = RICH_ENOMEM;
    if (st == RICH_OK &&
        (hipMemcpyAsync(dks, R.ks.data(), N * sizeof(double), hipMemcpyHostToDevice, stream) != hipSuccess ||
         hipMemcpyAsync(dp, R.p.data(), N * sizeof(double), hipMemcpyHostToDevice, stream) != hipSuccess ||
         hipStreamSynchronize(stream) != hipSuccess))
        st = RICH_EHIP;
    if (st == RICH_OK && R.after && hipStreamWaitEvent(stream, R.after, 0) != hipSuccess) st = RICH_EHIP;
    if (st == RICH_OK) st = rich_create(&R.prob, &R.opts, dks, stream, &h);
    if (st == RICH_OK && S->fused) st = batcher ? rich::batcher_attach(h, batcher) : RICH_EHIP;
    if (st == RICH_OK) st = rich_set_state(h, dp);
    rich_status warn = RICH_OK;  // largest warning of a completed step
    for (int t = 0; t < R.nsteps && st >= 0; t++) {
        double t0 = wall_s();
        rich_step_stats_t ss;
        st = rich_step(h, 1, &ss);
        R.step_ms.push_back(1e3 * (wall_s() - t0));
        R.stats.push_back(ss);
        if (st > warn) warn = st;
    }
    if (st >= 0) st = warn;
    if (h) {
        rich_status g = rich_get_state(h, dp);
        if (g == RICH_OK && hipMemcpyAsync(R.p.data(), dp, N * sizeof(double), hipMemcpyDeviceToHost, stream) == hipSuccess)
            (void)hipStreamSynchronize(stream);
        rich_destroy(h);
    }
    if (dks) (void)hipFree(dks);
    if (dp) (void)hipFree(dp);
    if (R.after) {
        (void)hipEventDestroy(R.after);
        R.after = nullptr;
    }
    R.result = st;
}

void worker_main(rich_server *S) {
    (void)hipSetDevice(S->device);
    hipStream_t stream = nullptr;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) return;
    for (;;) {
        std::shared_ptr<Request> R;
        rich_batcher *batcher = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            // FIFO: the head of the queue is admitted once its plan fits the budget
            S->cv.wait(lk, [&] { return S->stop || (!S->queue.empty() && S->queue.front()->bytes <= S->budget - S->in_use); });
            if (S->stop) break;
            R = S->queue.front();
            S->queue.pop_front();
            S->in_use += R->bytes;
            S->running++;
            if (S->fused) {
                rich_batcher *&b = S->batchers[batch_class(*R)];
                if (!b) b = rich::batcher_create(S->fused == 2);
                batcher = b;
            }
            R->state = RICH_REQ_RUNNING;
            R->t_start = wall_s();
        }
        run_request(S, stream, *R, batcher);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            R->t_end = wall_s();
            R->state = RICH_REQ_DONE;
            S->in_use -= R->bytes;
            S->running--;
        }
        S->cv.notify_all();
    }
    (void)hipStreamDestroy(stream);
}

}  // namespace

extern "C" {

rich_status rich_server_create(size_t hbm_budget, int max_active, void *hip_stream, rich_server_t *out) {
    if (!out || hbm_budget == 0 || max_active < 1 || max_active > 64) return RICH_EINVAL;
    int device = 0;
    if (hip_stream) {
        HIP_TRY(hipStreamGetDevice((hipStream_t)hip_stream, &device));
    } else if (hipGetDevice(&device) != hipSuccess) {
        (void)hipGetLastError();
        device = 0;
    }
    rich_server *S = new rich_server();
    S->budget = hbm_budget;
    S->device = device;
    S->order = (hipStream_t)hip_stream;
    for (int t = 0; t < max_active; t++) S->workers.emplace_back(worker_main, S);
    *out = S;
    return RICH_OK;
}

rich_status rich_server_submit(rich_server_t S, const rich_problem_t *prob, const rich_solver_opts_t *opts,
                               const double *Ks_host, const double *p0_host, int nsteps, int64_t *req_id) {
    if (!S || !prob || !opts || !Ks_host || !p0_host || nsteps < 0 || !req_id) return RICH_EINVAL;
    size_t bytes = 0;
    RICH_TRY(rich_query_bytes(prob, opts, &bytes));
    int64_t N = (int64_t)prob->nx * prob->ny * prob->nz;
    bytes += 2 * (size_t)N * sizeof(double);  // staging of K_s and p
    if (bytes > S->budget) return RICH_EBUDGET;
    auto R = std::make_shared<Request>();
    R->prob = *prob;
    R->opts = *opts;
    R->ks.assign(Ks_host, Ks_host + N);
    R->p.assign(p0_host, p0_host + N);
    R->nsteps = nsteps;
    R->bytes = bytes;
    R->t_submit = wall_s();
    if (S->order) {
        HIP_TRY(hipEventCreateWithFlags(&R->after, hipEventDisableTiming));
        HIP_TRY(hipEventRecord(R->after, S->order));
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) {
            if (R->after) (void)hipEventDestroy(R->after);
            return RICH_ESTATE;
        }
        R->id = S->next_id++;
        S->all[R->id] = R;
        S->queue.push_back(R);
    }
    S->cv.notify_all();
    *req_id = R->id;
    return RICH_OK;
}

rich_status rich_server_poll(rich_server_t S, int64_t req_id, int *state, rich_status *result, double *p_host,
                             rich_step_stats_t *stats_host, double *step_ms_host, double *times_host) {
    if (!S || !state) return RICH_EINVAL;
    std::shared_ptr<Request> R;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->all.find(req_id);
        if (it == S->all.end()) return RICH_EINVAL;
        R = it->second;
        *state = R->state;
    }
    if (*state != RICH_REQ_DONE) return RICH_OK;
    if (result) *result = R->result;
    if (p_host) memcpy(p_host, R->p.data(), R->p.size() * sizeof(double));
    for (size_t t = 0; t < R->stats.size(); t++) {
        if (stats_host) stats_host[t] = R->stats[t];
        if (step_ms_host) step_ms_host[t] = R->step_ms[t];
    }
    if (times_host) {
        times_host[0] = R->t_start - R->t_submit;  // admission wait [s]
        times_host[1] = R->t_end - R->t_start;     // resident time [s]
        times_host[2] = (double)R->stats.size();   // steps run
    }
    return RICH_OK;
}

rich_status rich_server_set_batching(rich_server_t S, int mode) {
    if (!S || mode < 0 || mode > 2) return RICH_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->next_id != 1) return RICH_ESTATE;
    S->fused = mode;
    return RICH_OK;
}

rich_status rich_server_batch_stats(rich_server_t S, int64_t *flushes, int64_t *products) {
    if (!S) return RICH_EINVAL;
    int64_t f = 0, p = 0;
    std::lock_guard<std::mutex> lk(S->mu);
    for (auto &kv : S->batchers) {
        int64_t f1 = 0, p1 = 0;
        if (kv.second) rich::batcher_stats(kv.second, &f1, &p1);
        f += f1;
        p += p1;
    }
    if (flushes) *flushes = f;
    if (products) *products = p;
    return RICH_OK;
}

rich_status rich_server_run_until_idle(rich_server_t S) {
    if (!S) return RICH_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv.wait(lk, [&] { return S->queue.empty() && S->running == 0; });
    return RICH_OK;
}

rich_status rich_server_destroy(rich_server_t S) {
    if (!S) return RICH_EINVAL;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv.wait(lk, [&] { return S->running == 0; });  // let running simulations finish
        S->stop = true;
        for (auto &R : S->queue) {
            R->state = RICH_REQ_DONE;
            R->result = RICH_ESTATE;  // never admitted
            if (R->after) {
                (void)hipEventDestroy(R->after);
                R->after = nullptr;
            }
        }
        S->queue.clear();
    }
    S->cv.notify_all();
    for (auto &t : S->workers) t.join();
    for (auto &kv : S->batchers) rich::batcher_destroy(kv.second);
    delete S;
    return RICH_OK;
}

}  // extern "C"
