// Request server of libfciqmc: continuous batching of FCIQMC solves on one
// device, written against the library's public C ABI.
//
// Requests (a system, run parameters, a convergence check interval and a
// step cap) queue in arrival order.  Each poll step admits queued requests
// while the head fits the device-memory budget and the running-set limit,
// advances every running request by one step in one batch (one set of
// launches for all of them), checks each request's energy report on its own
// step clock, and retires converged or capped requests, which frees their
// slot and reservation for the next admission.  A request's trajectory is
// that of the same run stepped alone, so its result does not depend on what
// else is running.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <memory>
#include <vector>

#include "../../include/fciqmc.h"
#include "errors.hpp"

namespace {

struct Request {
    const fciqmc_system* sys = nullptr;
    fciqmc_params p{};
    int interval = 100;
    int64_t max_steps = 0;
    fciqmc_run* run = nullptr;
    fciqmc_request_info info{};
};

}  // namespace

struct fciqmc_server {
    int64_t budget = 0;
    int max_running = 0;
    void* stream = nullptr;
    fciqmc_batch* batch = nullptr;
    std::vector<std::unique_ptr<Request>> all;  // indexed by ticket
    std::deque<Request*> queue;
    std::vector<Request*> running;              // in the batch's member order
    int64_t reserved = 0;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }

    ~fciqmc_server() {
        for (Request* q : running) fciqmc_free_run(q->run);
        if (batch) fciqmc_batch_free(batch);
    }

    void finish(Request* q, int state, int error) {
        q->info.state = state;
        q->info.error = error;
        q->info.t_done = now();
        if (q->run) {
            fciqmc_free_run(q->run);  // leaves the batch
            q->run = nullptr;
        }
        reserved -= q->info.reserved_bytes;
        running.erase(std::find(running.begin(), running.end(), q));
    }

    // Admit from the head of the queue while it fits (first come, first served).
    int admit() {
        while (!queue.empty() && (int)running.size() < max_running) {
            Request* q = queue.front();
            const int64_t need = q->info.reserved_bytes;
            if (need > budget) {  // can never fit
                queue.pop_front();
                q->info.state = FCIQMC_REQ_FAILED;
                q->info.error = FCIQMC_ENOMEM;
                q->info.t_done = now();
                continue;
            }
            if (reserved + need > budget) break;
            queue.pop_front();
            fciqmc_params p = q->p;
            if (p.hbm_budget_bytes <= 0 || p.hbm_budget_bytes > need) p.hbm_budget_bytes = need;
            q->info.t_admit = now();
            int rc = fciqmc_init(q->sys, &p, stream, &q->run);
            if (rc == 0) {
                rc = fciqmc_batch_add(batch, q->run);
                if (rc) {
                    fciqmc_free_run(q->run);
                    q->run = nullptr;
                }
            }
            if (rc) {
                q->info.state = FCIQMC_REQ_FAILED;
                q->info.error = rc;
                q->info.t_done = now();
                continue;
            }
            q->info.state = FCIQMC_REQ_RUNNING;
            reserved += need;
            running.push_back(q);
        }
        return 0;
    }

    // One batch step of every running request, then checks and retirements.
    int step() {
        const size_t m = running.size();
        std::vector<fciqmc_step_stats> row(m);
        std::memset(row.data(), 0, sizeof(fciqmc_step_stats) * m);
        const int rc = fciqmc_batch_step(batch, 1, row.data());
        std::vector<Request*> done, failed;
        for (size_t i = 0; i < m; ++i) {
            Request* q = running[i];
            if (row[i].iter != q->info.steps + 1) {  // this member did not record the step
                failed.push_back(q);
                continue;
            }
            q->info.steps = row[i].iter;
            q->info.attempts += row[i].attempts;
            const bool cap = q->info.steps >= q->max_steps;
            if (q->info.steps % q->interval == 0 || cap) {
                fciqmc_energy(q->run, &q->info.energy);
                q->info.converged = q->info.energy.converged;
                if (q->info.converged || cap) done.push_back(q);
            }
        }
        for (Request* q : failed) finish(q, FCIQMC_REQ_FAILED, rc ? rc : FCIQMC_EDEVICE);
        for (Request* q : done) finish(q, FCIQMC_REQ_DONE, 0);
        return 0;
    }
};

extern "C" {

int64_t fciqmc_estimate_bytes(const fciqmc_system* sys, const fciqmc_params* p);

int fciqmc_server_create(int64_t hbm_budget_bytes, int max_running, void* stream, fciqmc_server** out) {
    if (!out) return fq_set_error(FCIQMC_EINVAL, "null argument");
    *out = nullptr;
    if (hbm_budget_bytes <= 0) return fq_set_error(FCIQMC_EINVAL, "the device-memory budget must be positive");
    if (max_running < 1) return fq_set_error(FCIQMC_EINVAL, "max_running must be >= 1");
    std::unique_ptr<fciqmc_server> s(new fciqmc_server());
    s->budget = hbm_budget_bytes;
    s->max_running = max_running;
    s->stream = stream;
    const int rc = fciqmc_batch_create(stream, &s->batch);
    if (rc) return rc;
    *out = s.release();
    return 0;
}

int fciqmc_server_submit(fciqmc_server* srv, const fciqmc_system* sys, const fciqmc_params* p, int check_interval,
                         int64_t max_steps, double t_arrival, int64_t* ticket) {
    if (!srv || !sys || !p || !ticket) return fq_set_error(FCIQMC_EINVAL, "null argument");
    if (check_interval < 1) return fq_set_error(FCIQMC_EINVAL, "check_interval must be >= 1");
    if (max_steps < 1) return fq_set_error(FCIQMC_EINVAL, "max_steps must be >= 1");
    const int64_t need = fciqmc_estimate_bytes(sys, p);
    if (need < 0) return (int)need;
    std::unique_ptr<Request> q(new Request());
    q->sys = sys;
    q->p = *p;
    q->interval = check_interval;
    q->max_steps = max_steps;
    q->info.state = FCIQMC_REQ_QUEUED;
    q->info.reserved_bytes = need;
    q->info.t_arrival = t_arrival >= 0.0 ? t_arrival : srv->now();
    q->info.t_admit = q->info.t_done = -1.0;
    for (double* e : {&q->info.energy.e_proj, &q->info.energy.e_proj_err, &q->info.energy.shift,
                      &q->info.energy.shift_err})
        *e = -1.0;
    *ticket = (int64_t)srv->all.size();
    srv->queue.push_back(q.get());
    srv->all.push_back(std::move(q));
    return 0;
}

int fciqmc_server_poll(fciqmc_server* srv, int n_steps, int* n_running, int* n_queued) {
    if (!srv) return fq_set_error(FCIQMC_EINVAL, "null argument");
    if (n_steps < 0) return fq_set_error(FCIQMC_EINVAL, "n_steps must be >= 0");
    int rc = srv->admit();
    for (int i = 0; i < n_steps && rc == 0 && !srv->running.empty(); ++i) {
        rc = srv->step();
        if (rc == 0) rc = srv->admit();
    }
    if (n_running) *n_running = (int)srv->running.size();
    if (n_queued) *n_queued = (int)srv->queue.size();
    return rc;
}

int fciqmc_server_info(const fciqmc_server* srv, int64_t ticket, fciqmc_request_info* out) {
    if (!srv || !out) return fq_set_error(FCIQMC_EINVAL, "null argument");
    if (ticket < 0 || ticket >= (int64_t)srv->all.size()) return fq_set_error(FCIQMC_EINVAL, "unknown ticket");
    *out = srv->all[(size_t)ticket]->info;
    return 0;
}

double fciqmc_server_clock(const fciqmc_server* srv) { return srv ? srv->now() : 0.0; }

void fciqmc_server_free(fciqmc_server* srv) { delete srv; }

}  // extern "C"
