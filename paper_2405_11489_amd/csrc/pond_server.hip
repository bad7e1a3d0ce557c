// pond_server.hip -- continuous-batching server of PonD requests.
//
// Requests (parameters, initial fields, step count) are queued first in, first
// out.  A worker thread admits the head of the queue whenever its state
// footprint (pond_state_bytes) fits the HBM budget next to the admitted
// requests.  Each round steps, through one pond_batch, the admitted requests
// with the least remaining work (nodes x steps) -- of one lattice, precision,
// stencil and energy split, those of the request with the least -- as many as
// it takes to hold fill_nodes nodes
// (enough tiles to fill the chip): small requests finish
// together at full-chip throughput instead of at the pace of the largest
// co-runner, and large ones absorb the remaining capacity.  The queue is
// re-examined every chunk_steps steps and as soon as a request finishes.  A finished request's moments (and, on request, its raw state)
// are copied to host memory and its device memory is released, which may
// admit the next queued request.  Because a batch member's results equal the
// instance's results alone, a request's output does not depend on the
// traffic it was served with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "pond_ctx.h"

using namespace pond;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    int64_t id;
    pond_params p;
    int64_t steps_total;
    int64_t steps_done = 0;
    int32_t flags;
    int32_t state = POND_REQ_QUEUED;
    pond_status error = POND_OK;
    std::vector<double> fields;  // rho, ux, uy, T until admission
    std::vector<double> moments; // rho, ux, uy, T, p after completion (flag)
    std::vector<double> raw;     // f (16 N), g (16 N), frame (3 N), u_ref (2) (flag)
    size_t bytes = 0;
    double t_submit = 0, t_admit = -1, t_done = -1;
    pond_ctx *ctx = nullptr;
};

}  // namespace

struct pond_server {
    pond_server_config cfg;
    int device;
    hipStream_t stream;
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<int64_t> queue;
    std::map<int64_t, std::unique_ptr<Request>> reqs;
    std::vector<Request *> running;  // worker thread only
    size_t used_bytes = 0;           // footprint of admitted, unfinished requests
    int64_t next_id = 1;
    int64_t outstanding = 0;         // queued + running
    bool stop = false;
    pond_server_stats_t stats{};
    std::thread worker;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

int64_t nodes_of(const pond_params &p) { return int64_t(p.nx) * p.ny; }

// Worker side: create, initialise and (optionally) tune a request's context.
pond_status admit(pond_server *s, Request *r) {
    pond_status st = pond_create(&r->p, s->stream, nullptr, 0, &r->ctx);
    if (st != POND_OK) return st;
    const int64_t N = nodes_of(r->p);
    const double *f = r->fields.data();
    st = pond_init_fields(r->ctx, f, f + N, f + 2 * N, f + 3 * N);
    if (st == POND_OK && s->cfg.autotune_steps > 0) {
        pond_tuning t;
        if (!tuning_cache_lookup(r->ctx, &t)) st = pond_autotune(r->ctx, int(s->cfg.autotune_steps), nullptr);
    }
    if (st != POND_OK) {
        (void)pond_destroy(r->ctx);
        r->ctx = nullptr;
    }
    return st;
}

// Worker side: copy the requested outputs of a finished member to the host.
pond_status collect(Request *r) {
    const int64_t N = nodes_of(r->p);
    pond_status st = POND_OK;
    if (r->flags & POND_REQ_KEEP_MOMENTS) {
        r->moments.assign(size_t(5 * N), 0.0);
        double *m = r->moments.data();
        st = pond_moments(r->ctx, m, m + N, m + 2 * N, m + 3 * N, m + 4 * N);
    }
    if (st == POND_OK && (r->flags & POND_REQ_KEEP_STATE)) {
        // f (Q N), g (Q N), frame (3 N), u_ref (2): Q = 16 on D2Q16, 25 on D2Q25
        const int64_t Q = r->p.lattice;
        r->raw.assign(size_t((2 * Q + 3) * N + 2), 0.0);
        double *x = r->raw.data();
        st = pond_export_state(r->ctx, x, x + Q * N, x + 2 * Q * N, x + (2 * Q + 3) * N);
    }
    return st;
}

void worker_loop(pond_server *s) {
    (void)hipSetDevice(s->device);
    pond_batch *batch = nullptr;
    std::vector<Request *> current;  // members of batch
    bool dirty = true;               // selection changed since the batch was built
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // admission: strict FIFO under the HBM budget and the member cap (a
        // request never exceeds the budget alone, so an idle server admits it)
        while (!s->queue.empty()) {
            Request *r = s->reqs[s->queue.front()].get();
            const bool fits = s->used_bytes + r->bytes <= size_t(s->cfg.hbm_budget_bytes);
            const bool room = s->cfg.max_members <= 0 || int(s->running.size()) < s->cfg.max_members;
            if (!fits || !room) {
                ++s->stats.admission_waits;
                break;
            }
            s->queue.pop_front();
            s->used_bytes += r->bytes;
            lk.unlock();
            const double ta = s->now();
            pond_status st = admit(s, r);
            const double tb = s->now();
            lk.lock();
            s->stats.ns_admit += int64_t((tb - ta) * 1e9);
            r->fields.clear();
            r->fields.shrink_to_fit();
            if (st != POND_OK) {
                r->state = POND_REQ_FAILED;
                r->error = st;
                r->t_done = s->now();
                s->used_bytes -= r->bytes;
                --s->outstanding;
                ++s->stats.failed;
                s->cv_done.notify_all();
                continue;
            }
            r->state = POND_REQ_RUNNING;
            r->t_admit = s->now();
            s->running.push_back(r);
            ++s->stats.admitted;
        }
        if (s->running.empty()) {
            if (s->stop) break;
            s->cv_work.wait(lk, [s] { return s->stop || !s->queue.empty(); });
            continue;
        }
        // one round of batched steps.  Selection: the running requests with the
        // least remaining work (nodes x steps) first, adding requests until the
        // round holds fill_nodes nodes (enough tiles to fill the chip); with
        // fill_nodes <= 0 every running request steps.
        std::vector<Request *> run = s->running;
        if (s->cfg.fill_nodes > 0) {
            std::stable_sort(run.begin(), run.end(), [](const Request *a, const Request *b) {
                return nodes_of(a->p) * (a->steps_total - a->steps_done) <
                       nodes_of(b->p) * (b->steps_total - b->steps_done);
            });
        }
        // a batch runs one lattice, precision, stencil and split: those of the
        // first request in this order
        const pond_params &p0 = run.front()->p;
        const auto other = [&p0](const Request *r) {
            return r->p.lattice != p0.lattice || r->p.precision != p0.precision ||
                   r->p.interp_points != p0.interp_points || r->p.split != p0.split;
        };
        run.erase(std::remove_if(run.begin(), run.end(), other), run.end());
        if (s->cfg.fill_nodes > 0) {
            int64_t nodes = 0;
            size_t take = 0;
            while (take < run.size() && nodes < s->cfg.fill_nodes) nodes += nodes_of(run[take++]->p);
            run.resize(take);
            std::sort(run.begin(), run.end(), [](const Request *a, const Request *b) { return a->id < b->id; });
        }
        if (run != current) dirty = true;
        int64_t k = INT64_MAX;
        for (Request *r : run) k = std::min(k, r->steps_total - r->steps_done);
        if (s->cfg.chunk_steps > 0) k = std::min<int64_t>(k, s->cfg.chunk_steps);
        lk.unlock();
        const double t_round = s->now();
        pond_status st = POND_OK;
        if (dirty || !batch) {
            if (batch) (void)pond_batch_destroy(batch);
            batch = nullptr;
            std::vector<pond_ctx *> ctxs;
            for (Request *r : run) ctxs.push_back(r->ctx);
            st = pond_batch_create(ctxs.data(), int(ctxs.size()), s->stream, &batch);
            if (st == POND_OK) ++s->stats.batch_builds;
            current = run;
            dirty = false;
        }
        const double t_built = s->now();
        if (st == POND_OK && k > 0) st = pond_batch_step(batch, k);
        pond_status sync = st == POND_OK ? pond_batch_synchronize(batch) : st;
        const double t_stepped = s->now();
        // retire finished and failed members
        std::vector<Request *> finished;
        for (Request *r : run) {
            if (st == POND_OK) r->steps_done += k;
            if (r->ctx->failed || st != POND_OK || r->steps_done >= r->steps_total) finished.push_back(r);
        }
        std::vector<pond_status> outcome(finished.size(), POND_OK);
        for (size_t j = 0; j < finished.size(); ++j) {
            Request *r = finished[j];
            if (st != POND_OK)
                outcome[j] = st;
            else if (r->ctx->failed)
                outcome[j] = r->ctx->fail_status;
            else
                outcome[j] = collect(r);
        }
        if (!finished.empty() && batch) {
            (void)pond_batch_destroy(batch);
            batch = nullptr;
            current.clear();
        }
        for (Request *r : finished) {
            (void)pond_destroy(r->ctx);
            r->ctx = nullptr;
        }
        (void)sync;
        const double t_retired = s->now();
        lk.lock();
        s->stats.ns_build += int64_t((t_built - t_round) * 1e9);
        s->stats.ns_step += int64_t((t_stepped - t_built) * 1e9);
        s->stats.ns_retire += int64_t((t_retired - t_stepped) * 1e9);
        ++s->stats.rounds;
        s->stats.batched_steps += k;
        for (Request *r : run) s->stats.node_updates += (st == POND_OK ? k : 0) * nodes_of(r->p);
        for (size_t j = 0; j < finished.size(); ++j) {
            Request *r = finished[j];
            r->t_done = s->now();
            r->state = outcome[j] == POND_OK ? POND_REQ_DONE : POND_REQ_FAILED;
            r->error = outcome[j];
            if (outcome[j] != POND_OK) ++s->stats.failed;
            else ++s->stats.completed;
            s->used_bytes -= r->bytes;
            --s->outstanding;
            s->running.erase(std::find(s->running.begin(), s->running.end(), r));
            dirty = true;
        }
        if (!finished.empty()) s->cv_done.notify_all();
    }
    lk.unlock();
    if (batch) (void)pond_batch_destroy(batch);
}

}  // namespace

pond_status pond_server_config_default(pond_server_config *c) {
    if (!c) return fail(POND_ERR_INVALID_ARG, "config is NULL");
    std::memset(c, 0, sizeof *c);
    c->struct_size = sizeof(pond_server_config);
    c->hbm_budget_bytes = int64_t(64) << 30;
    c->max_members = 0;
    c->chunk_steps = 64;
    c->fill_nodes = int64_t(1) << 19;
    c->autotune_steps = 0;
    c->precision = POND_PREC_FP32;
    c->interp_points = 4;
    c->split = POND_SPLIT_TOTAL;
    return POND_OK;
}

pond_status pond_server_create(const pond_server_config *cfg, pond_server **out) {
    if (!out) return fail(POND_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!cfg || cfg->struct_size != sizeof(pond_server_config))
        return fail(POND_ERR_INVALID_ARG, "config is NULL or has the wrong struct_size");
    if (cfg->hbm_budget_bytes <= 0) return fail(POND_ERR_INVALID_ARG, "hbm_budget_bytes must be > 0");
    // -1 (POND_SERVE_ANY): requests of any value, batched apart
    if (cfg->precision != POND_PREC_FP32 && cfg->precision != POND_PREC_FP64 &&
        cfg->precision != POND_SERVE_ANY)
        return fail(POND_ERR_INVALID_ARG, "unknown precision %d", cfg->precision);
    if (cfg->interp_points != 3 && cfg->interp_points != 4 &&
        cfg->interp_points != POND_SERVE_ANY)
        return fail(POND_ERR_INVALID_ARG, "interp_points must be 3 or 4");
    if (cfg->split != POND_SPLIT_TOTAL && cfg->split != POND_SPLIT_INTERNAL &&
        cfg->split != POND_SPLIT_NONTRANS && cfg->split != POND_SERVE_ANY)
        return fail(POND_ERR_INVALID_ARG, "unknown split %d", cfg->split);
    if (cfg->chunk_steps < 0 || cfg->autotune_steps < 0)
        return fail(POND_ERR_INVALID_ARG, "chunk_steps and autotune_steps must be >= 0");
    pond_server *s = new (std::nothrow) pond_server();
    if (!s) return fail(POND_ERR_OUT_OF_MEMORY, "host allocation failed");
    s->cfg = *cfg;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipStreamCreate(&s->stream);
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "server stream");
    }
    s->t0 = Clock::now();
    try {
        s->worker = std::thread(worker_loop, s);
    } catch (...) {
        (void)hipStreamDestroy(s->stream);
        delete s;
        return fail(POND_ERR_OUT_OF_MEMORY, "worker thread");
    }
    *out = s;
    return POND_OK;
}

pond_status pond_server_submit(pond_server *s, const pond_params *p, const double *rho,
                               const double *ux, const double *uy, const double *T, int64_t nsteps,
                               int32_t flags, int64_t *id) {
    if (!s || !p || !rho || !ux || !uy || !T || !id)
        return fail(POND_ERR_INVALID_ARG, "NULL argument");
    if (nsteps < 0) return fail(POND_ERR_INVALID_ARG, "nsteps < 0");
    if (flags & ~(POND_REQ_KEEP_MOMENTS | POND_REQ_KEEP_STATE))
        return fail(POND_ERR_INVALID_ARG, "unknown flags 0x%x", unsigned(flags));
    const size_t bytes = pond_state_bytes(p);
    if (bytes == 0) return fail(POND_ERR_INVALID_ARG, "invalid parameters: %s", last_error());
    const auto differs = [](int32_t v, int32_t c) { return c != POND_SERVE_ANY && v != c; };
    if (differs(p->precision, s->cfg.precision) ||
        differs(p->interp_points, s->cfg.interp_points) || differs(p->split, s->cfg.split))
        return fail(POND_ERR_INVALID_ARG,
                    "request precision / interp_points / split differ from the server's "
                    "(%d / %d / %d)",
                    s->cfg.precision, s->cfg.interp_points, s->cfg.split);
    if (bytes > size_t(s->cfg.hbm_budget_bytes))
        return fail(POND_ERR_INVALID_ARG, "request needs %zu bytes, above the budget of %lld", bytes,
                    (long long)s->cfg.hbm_budget_bytes);
    auto r = std::unique_ptr<Request>(new (std::nothrow) Request());
    if (!r) return fail(POND_ERR_OUT_OF_MEMORY, "host allocation failed");
    const int64_t N = nodes_of(*p);
    try {
        r->fields.resize(size_t(4 * N));
    } catch (...) {
        return fail(POND_ERR_OUT_OF_MEMORY, "host copy of the fields");
    }
    std::memcpy(r->fields.data(), rho, size_t(N) * sizeof(double));
    std::memcpy(r->fields.data() + N, ux, size_t(N) * sizeof(double));
    std::memcpy(r->fields.data() + 2 * N, uy, size_t(N) * sizeof(double));
    std::memcpy(r->fields.data() + 3 * N, T, size_t(N) * sizeof(double));
    r->p = *p;
    r->steps_total = nsteps;
    r->flags = flags;
    r->bytes = bytes;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(POND_ERR_STATE, "server is shutting down");
    r->id = s->next_id++;
    r->t_submit = s->now();
    *id = r->id;
    s->queue.push_back(r->id);
    s->reqs[r->id] = std::move(r);
    ++s->outstanding;
    ++s->stats.submitted;
    s->cv_work.notify_one();
    return POND_OK;
}

pond_status pond_server_poll(pond_server *s, int64_t id, pond_request_info *out) {
    if (!s || !out) return fail(POND_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(POND_ERR_INVALID_ARG, "unknown request %lld", (long long)id);
    const Request &r = *it->second;
    out->state = r.state;
    out->error = r.error;
    out->steps_done = r.steps_done;
    out->steps_total = r.steps_total;
    out->state_bytes = int64_t(r.bytes);
    out->t_submit = r.t_submit;
    out->t_admit = r.t_admit;
    out->t_done = r.t_done;
    return POND_OK;
}

pond_status pond_server_wait(pond_server *s, int64_t id) {
    if (!s) return fail(POND_ERR_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    if (id == 0) {
        s->cv_done.wait(lk, [s] { return s->outstanding == 0; });
        return POND_OK;
    }
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(POND_ERR_INVALID_ARG, "unknown request %lld", (long long)id);
    Request *r = it->second.get();
    s->cv_done.wait(lk, [r] { return r->state == POND_REQ_DONE || r->state == POND_REQ_FAILED; });
    return POND_OK;
}

pond_status pond_server_result(pond_server *s, int64_t id, double *moments, double *state) {
    if (!s) return fail(POND_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(POND_ERR_INVALID_ARG, "unknown request %lld", (long long)id);
    const Request &r = *it->second;
    if (r.state == POND_REQ_FAILED)
        return fail(r.error == POND_OK ? POND_ERR_STATE : r.error, "request %lld failed",
                    (long long)id);
    if (r.state != POND_REQ_DONE) return fail(POND_ERR_STATE, "request %lld is not finished", (long long)id);
    if (moments) {
        if (!(r.flags & POND_REQ_KEEP_MOMENTS))
            return fail(POND_ERR_INVALID_ARG, "request %lld kept no moments", (long long)id);
        std::memcpy(moments, r.moments.data(), r.moments.size() * sizeof(double));
    }
    if (state) {
        if (!(r.flags & POND_REQ_KEEP_STATE))
            return fail(POND_ERR_INVALID_ARG, "request %lld kept no state", (long long)id);
        std::memcpy(state, r.raw.data(), r.raw.size() * sizeof(double));
    }
    return POND_OK;
}

pond_status pond_server_release(pond_server *s, int64_t id) {
    if (!s) return fail(POND_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(POND_ERR_INVALID_ARG, "unknown request %lld", (long long)id);
    if (it->second->state != POND_REQ_DONE && it->second->state != POND_REQ_FAILED)
        return fail(POND_ERR_STATE, "request %lld is not finished", (long long)id);
    s->reqs.erase(it);
    return POND_OK;
}

pond_status pond_server_get_stats(pond_server *s, pond_server_stats_t *out) {
    if (!s || !out) return fail(POND_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->queued = int64_t(s->queue.size());
    out->running = int64_t(s->running.size());
    out->used_bytes = int64_t(s->used_bytes);
    return POND_OK;
}

pond_status pond_server_destroy(pond_server *s) {
    if (!s) return POND_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        // queued requests are dropped; running ones finish
        for (int64_t id : s->queue) {
            Request *r = s->reqs[id].get();
            r->state = POND_REQ_FAILED;
            r->error = POND_ERR_STATE;
            --s->outstanding;
        }
        s->queue.clear();
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    hipError_t e = hipStreamDestroy(s->stream);
    delete s;
    return e == hipSuccess ? POND_OK : hip_fail(e, "hipStreamDestroy");
}
