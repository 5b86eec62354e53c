// Eigensolver server: continuous batching of independent two-level BPJD solves on
// one GPU.
//
// Each request is a complete problem (K, M, decomposition, options) solved by
// Algorithm 3.1.  Requests are admitted in arrival order as solve slots and device
// memory (the HBM budget) free up; every admitted solve owns a slot with its own
// non-blocking HIP stream, and the solves of all slots advance together, so the
// kernels of different requests overlap on the device and the host-side stop test
// of one request never stalls another.
//
// Host threads:
//   plan   - (kPlanners of them) plan queued requests on the host, in submission
//            order, a few ahead of admission: validation, subdomains, band layout,
//            device footprint;
//   admit  - takes the oldest queued request once it is planned, waits until a slot
//            is free and its footprint fits the budget, then allocates, uploads and
//            enqueues its setup;
//   step   - polls the read-back event of every running solve and enqueues its
//            next stage as soon as that event has completed;
//   reap   - copies finished results to host memory, frees the device memory and
//            returns the slot and the bytes to the admission test.
// A request's result is the same whether it runs alone or in a mix: its kernels,
// launch shapes and reduction orders do not depend on what else runs.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <memory>
#include <unordered_map>

#include "common.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Request {
    uint64_t id = 0;
    // host copies of the inputs (borrowed arrays are copied at submission)
    std::vector<int32_t> Kptr, Kcol, Mptr, Mcol, Pptr, Pcol, sub_ptr, sub_idx;
    std::vector<double> Kval, Mval, Pval, coords, cx, cy, X_init;
    bpjd_csr K{}, M{};
    bpjd_dd dd{};
    bpjd_dd_geom geom{};
    bool use_geom = false;
    bpjd_opts opts{};
    int n = 0, k = 0;

    enum State { QUEUED, RUNNING, DONE } state = QUEUED;
    int rc = BPJD_OK;
    std::string err;
    bool planned = false;                    // set by a planner
    int plan_rc = BPJD_OK;
    std::string plan_err;
    bpjd_problem* planned_p = nullptr;       // planned, not yet materialised
    bpjd_problem* p = nullptr;
    bpjd::SolveRun* run = nullptr;
    int slot = -1;
    size_t footprint = 0;
    std::vector<double> eigvals, eigvecs;
    bpjd_stats stats{};
    Clock::time_point t_submit, t_admit, t_done;
};

void copy_csr(const bpjd_csr& in, std::vector<int32_t>& ptr, std::vector<int32_t>& col, std::vector<double>& val,
              bpjd_csr& out) {
    const int64_t nnz = in.rowptr[in.n_rows];
    ptr.assign(in.rowptr, in.rowptr + in.n_rows + 1);
    col.assign(in.col, in.col + nnz);
    val.assign(in.val, in.val + nnz);
    out = in;
    out.nnz = nnz;
    out.rowptr = ptr.data();
    out.col = col.data();
    out.val = val.data();
    out.mem = BPJD_MEM_HOST;
}

}  // namespace

constexpr int kPlanners = 3;                 // host planning threads
constexpr int kPlanAhead = 4;                // planned requests waiting for admission, at most

struct bpjd_server {
    bpjd_ctx* ctx = nullptr;                 // caller's context: device
    size_t budget = 0;
    int max_slots = 0;
    std::vector<std::unique_ptr<bpjd_ctx>> slot_ctx;   // one non-blocking stream per slot
    bpjd::DevArena arena;                    // the whole budget, one device block, sub-allocated
    int arena_route = 0;                     // how the block was obtained: 0 hipMalloc, 1 the allocator
    std::vector<char> slot_busy;

    std::mutex mu;
    std::condition_variable cv_admit, cv_step, cv_reap, cv_plan;
    bool stopping = false;
    uint64_t next_id = 1;
    std::deque<Request*> queued;
    std::deque<Request*> to_plan;            // submitted, not yet taken by a planner
    int plan_pending = 0;                    // being planned, or planned and not admitted
    std::vector<Request*> running;           // owned by the step thread while RUNNING
    std::deque<Request*> finished;           // handed from step to reap
    std::unordered_map<uint64_t, Request*> all;
    size_t in_use = 0;
    bpjd_server_info info{};

    std::thread admit_thr, step_thr, reap_thr;
    std::vector<std::thread> plan_thr;
};

namespace {

void finish_request(bpjd_server* s, Request* r, int rc, const std::string& err) {
    // caller holds s->mu
    if (r->state == Request::QUEUED) r->t_admit = Clock::now();   // never admitted
    r->rc = rc;
    r->err = err;
    r->state = Request::DONE;
    r->t_done = Clock::now();
    s->info.completed++;
    if (rc < 0 && rc != BPJD_ERR_NOCONV) s->info.failed++;
}

void plan_loop(bpjd_server* s) {
    (void)hipSetDevice(s->ctx->device);
    for (;;) {
        Request* r = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_plan.wait(lk, [&] {
                return s->stopping || (!s->to_plan.empty() && s->plan_pending < kPlanAhead);
            });
            if (s->stopping) return;
            r = s->to_plan.front();
            s->to_plan.pop_front();
            s->plan_pending++;
        }
        bpjd_problem* p = nullptr;
        int rc = bpjd::plan_problem(s->ctx, &r->K, &r->M, r->use_geom ? nullptr : &r->dd,
                                    r->use_geom ? &r->geom : nullptr, &r->opts, &p);
        std::string err = rc < 0 ? bpjd_last_error(nullptr) : "";
        if (rc == BPJD_OK && p->footprint > s->budget) {
            rc = BPJD_ERR_OVER_BUDGET;
            err = "request needs " + std::to_string(p->footprint) + " device bytes, budget is " +
                  std::to_string(s->budget);
        }
        if (rc < 0 && p) {
            bpjd_problem_destroy(p);
            p = nullptr;
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            r->planned_p = p;
            r->plan_rc = rc;
            r->plan_err = err;
            r->planned = true;
        }
        s->cv_admit.notify_all();
    }
}

void admit_loop(bpjd_server* s) {
    (void)hipSetDevice(s->ctx->device);
    for (;;) {
        Request* r = nullptr;
        bpjd_problem* p = nullptr;
        int rc = BPJD_OK;
        std::string err;
        {
            // the oldest queued request, once a planner has finished with it
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_admit.wait(lk, [&] { return s->stopping || (!s->queued.empty() && s->queued.front()->planned); });
            if (s->stopping) return;
            r = s->queued.front();
            p = r->planned_p;
            rc = r->plan_rc;
            err = r->plan_err;
        }
        if (rc < 0) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->queued.pop_front();
            s->plan_pending--;
            finish_request(s, r, rc, err);
            r->stats.queue_ms = ms_between(r->t_submit, r->t_admit);
            r->stats.latency_ms = ms_between(r->t_submit, r->t_done);
            s->cv_plan.notify_one();
            continue;
        }
        // wait for a free slot and room in the budget: the footprint fits the bytes left, and
        // the blocks fit the server's block as it is now (first fit, so fragmentation can
        // delay a request; with nothing running the whole block is free and it fits)
        int slot = -1;
        const std::vector<size_t> blocks = bpjd::planned_blocks(p);
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_admit.wait(lk, [&] {
                if (s->stopping) return true;
                if (s->in_use + p->footprint > s->budget) return false;
                bool slot_free = false;
                for (int q = 0; q < s->max_slots; ++q) slot_free = slot_free || !s->slot_busy[q];
                // last: reserves the blocks when everything else allows admission
                return slot_free && s->arena.alloc_all(blocks, p->reserved);
            });
            if (s->stopping) return;        // the request (and its plan) is freed by destroy
            for (int q = 0; q < s->max_slots && slot < 0; ++q)
                if (!s->slot_busy[q]) slot = q;
            s->slot_busy[slot] = 1;
            s->in_use += p->footprint;
            s->info.peak_bytes = std::max<uint64_t>(s->info.peak_bytes, s->in_use);
            s->queued.pop_front();
            s->plan_pending--;
            r->planned_p = nullptr;
            s->cv_plan.notify_one();
            r->state = Request::RUNNING;
            r->t_admit = Clock::now();
        }
        p->reserved_bytes = blocks;
        r->slot = slot;
        r->footprint = p->footprint;
        r->p = p;
        p->ctx = s->slot_ctx[slot].get();
        rc = bpjd::materialize_problem(p);
        if (rc == BPJD_OK) rc = bpjd::run_create(p, &r->run);
        if (rc == BPJD_OK) rc = bpjd::run_begin(r->run);
        std::lock_guard<std::mutex> lk(s->mu);
        if (rc < 0) {
            r->err = bpjd_last_error(nullptr);
            r->rc = rc;
            s->finished.push_back(r);   // the reaper frees what was allocated
            s->cv_reap.notify_one();
        } else {
            s->running.push_back(r);
            s->info.peak_running = std::max<uint32_t>(s->info.peak_running, (uint32_t)s->running.size());
            s->cv_step.notify_one();
        }
    }
}

void step_loop(bpjd_server* s) {
    (void)hipSetDevice(s->ctx->device);
    std::vector<Request*> mine;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (mine.empty()) s->cv_step.wait(lk, [&] { return s->stopping || !s->running.empty(); });
            if (s->stopping) return;
            mine = s->running;
        }
        std::vector<Request*> done;
        for (Request* r : mine) {
            int q = bpjd::run_poll(r->run);
            if (q == 0) continue;
            if (q > 0) q = bpjd::run_advance(r->run);
            if (q == 0) continue;
            if (q < 0) {
                r->rc = q;
                r->err = bpjd_last_error(nullptr);
            }
            done.push_back(r);
        }
        if (!done.empty()) {
            std::lock_guard<std::mutex> lk(s->mu);
            for (Request* r : done) {
                s->running.erase(std::find(s->running.begin(), s->running.end(), r));
                s->finished.push_back(r);
            }
            s->cv_reap.notify_one();
            mine = s->running;
        } else {
            std::this_thread::yield();
        }
    }
}

void reap_loop(bpjd_server* s) {
    (void)hipSetDevice(s->ctx->device);
    for (;;) {
        Request* r = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_reap.wait(lk, [&] { return s->stopping || !s->finished.empty(); });
            if (s->stopping) return;
            r = s->finished.front();
            s->finished.pop_front();
        }
        int rc = r->rc;
        std::string err = r->err;
        if (rc == BPJD_OK) {
            r->eigvals.assign(r->k, 0.0);
            r->eigvecs.assign((size_t)r->n * r->k, 0.0);
            rc = bpjd::run_finish(r->run, r->eigvals.data(), r->eigvecs.data(), BPJD_MEM_HOST, &r->stats);
            if (rc < 0) err = bpjd_last_error(nullptr);
        }
        if (r->p) (void)hipStreamSynchronize(r->p->ctx->stream);
        bpjd::run_destroy(r->run);
        r->run = nullptr;
        bpjd_problem_destroy(r->p);
        r->p = nullptr;
        std::lock_guard<std::mutex> lk(s->mu);
        s->in_use -= r->footprint;
        s->slot_busy[r->slot] = 0;
        finish_request(s, r, rc, err);
        r->stats.queue_ms = ms_between(r->t_submit, r->t_admit);
        r->stats.latency_ms = ms_between(r->t_submit, r->t_done);
        s->cv_admit.notify_one();
    }
}

}  // namespace

extern "C" {

int bpjd_server_create(bpjd_ctx* ctx, size_t hbm_budget_bytes, int32_t max_slots, bpjd_server** out) {
    bpjd::CtxScope cs_(ctx);
    if (!ctx || !out) return bpjd::fail(BPJD_ERR_ARG, "NULL argument");
    if (max_slots < 1 || max_slots > 64) return bpjd::fail(BPJD_ERR_ARG, "max_slots must be in [1, 64]");
    BPJD_HIP(hipSetDevice(ctx->device));
    size_t free_b = 0, total_b = 0;
    BPJD_HIP(hipMemGetInfo(&free_b, &total_b));
    auto* s = new bpjd_server();
    s->ctx = ctx;
    s->budget = bpjd::DevArena::round(hbm_budget_bytes ? hbm_budget_bytes : free_b / 10 * 9);
    s->max_slots = max_slots;
    // the whole budget as one device block, from the context's allocator or hipMalloc:
    // admitting and reaping requests then sub-allocate and release without any device
    // allocation call (which would synchronise the device under running solves)
    void* block = nullptr;
    if (ctx->alloc.alloc) {
        block = ctx->alloc.alloc(s->budget, ctx->alloc.user);
        s->arena_route = 1;
    } else if (hipMalloc(&block, s->budget) != hipSuccess) {
        block = nullptr;
    }
    if (!block) {
        (void)hipGetLastError();
        delete s;
        return bpjd::fail(BPJD_ERR_OOM, "server block of " + std::to_string(hbm_budget_bytes) + " bytes");
    }
    s->arena.base = (char*)block;
    s->arena.size = s->budget;
    s->arena.free_[0] = s->budget;
    s->slot_busy.assign(max_slots, 0);
    int made = 0;
    for (int q = 0; q < max_slots; ++q) {
        auto c = std::make_unique<bpjd_ctx>();
        c->device = ctx->device;
        c->own_stream = true;
        c->arena = &s->arena;
        const bool ok = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) == hipSuccess &&
                        hipHostMalloc((void**)&c->hbuf, 4096 * sizeof(double)) == hipSuccess;
        s->slot_ctx.push_back(std::move(c));
        if (!ok) break;
        ++made;
    }
    if (made < max_slots) {
        for (auto& c : s->slot_ctx) {
            if (c->stream) (void)hipStreamDestroy(c->stream);
            if (c->hbuf) (void)hipHostFree(c->hbuf);
        }
        if (s->arena_route == 1) ctx->alloc.free(block, ctx->alloc.user);
        else (void)hipFree(block);
        delete s;
        return bpjd::fail(BPJD_ERR_HIP, "slot stream or pinned buffer creation failed");
    }
    s->info.budget_bytes = s->budget;
    s->info.max_slots = max_slots;
    for (int q = 0; q < kPlanners; ++q) s->plan_thr.emplace_back(plan_loop, s);
    s->admit_thr = std::thread(admit_loop, s);
    s->step_thr = std::thread(step_loop, s);
    s->reap_thr = std::thread(reap_loop, s);
    *out = s;
    return BPJD_OK;
}

int bpjd_server_submit(bpjd_server* s, const bpjd_csr* K, const bpjd_csr* M, const bpjd_dd* dd,
                       const bpjd_dd_geom* geom, const bpjd_opts* opts, uint64_t* req_id) {
    bpjd::CtxScope cs_(s ? s->ctx : nullptr);
    if (!s || !K || !M || !opts || !req_id || (!dd && !geom) || (dd && geom))
        return bpjd::fail(BPJD_ERR_ARG, "need K, M, opts, req_id and exactly one of dd / geom");
    if (K->mem != BPJD_MEM_HOST || M->mem != BPJD_MEM_HOST || (dd && dd->P.mem != BPJD_MEM_HOST))
        return bpjd::fail(BPJD_ERR_ARG, "served matrices must be host arrays");
    if (!K->rowptr || !K->col || !K->val || !M->rowptr || !M->col || !M->val || K->n_rows < 1 || M->n_rows < 1)
        return bpjd::fail(BPJD_ERR_ARG, "empty or NULL CSR array");
    if (opts->k < 1) return bpjd::fail(BPJD_ERR_ARG, "k must be >= 1");
    auto* r = new Request();
    r->n = K->n_rows;
    r->k = opts->k;
    copy_csr(*K, r->Kptr, r->Kcol, r->Kval, r->K);
    copy_csr(*M, r->Mptr, r->Mcol, r->Mval, r->M);
    r->opts = *opts;
    // served solves keep the caller's graphs option: admission and reaping sub-allocate
    // from the server's block, so no device-wide synchronisation overlaps a capture
    if (opts->n_init > 0 && opts->X_init) {
        r->X_init.assign(opts->X_init, opts->X_init + (size_t)r->n * opts->n_init);
        r->opts.X_init = r->X_init.data();
    }
    if (dd) {
        if (!dd->P.rowptr || !dd->P.col || !dd->P.val || !dd->sub_ptr || !dd->sub_idx || dd->n_sub < 1 ||
            dd->P.n_rows < 1) {
            delete r;
            return bpjd::fail(BPJD_ERR_DD, "incomplete decomposition");
        }
        copy_csr(dd->P, r->Pptr, r->Pcol, r->Pval, r->dd.P);
        r->sub_ptr.assign(dd->sub_ptr, dd->sub_ptr + dd->n_sub + 1);
        r->sub_idx.assign(dd->sub_idx, dd->sub_idx + std::max(0, r->sub_ptr.back()));
        r->dd.n_sub = dd->n_sub;
        r->dd.sub_ptr = r->sub_ptr.data();
        r->dd.sub_idx = r->sub_idx.data();
    } else {
        if (!geom->coords || !geom->cx || !geom->cy || geom->n_cx < 2 || geom->n_cy < 2) {
            delete r;
            return bpjd::fail(BPJD_ERR_ARG, "bad coarse grid");
        }
        r->use_geom = true;
        r->coords.assign(geom->coords, geom->coords + 2 * (size_t)r->n);
        r->cx.assign(geom->cx, geom->cx + geom->n_cx);
        r->cy.assign(geom->cy, geom->cy + geom->n_cy);
        r->geom = *geom;
        r->geom.coords = r->coords.data();
        r->geom.cx = r->cx.data();
        r->geom.cy = r->cy.data();
    }
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) {
        delete r;
        return bpjd::fail(BPJD_ERR_STATE, "server is shutting down");
    }
    r->id = s->next_id++;
    s->all[r->id] = r;
    s->queued.push_back(r);
    s->to_plan.push_back(r);
    s->info.submitted++;
    *req_id = r->id;
    s->cv_plan.notify_one();
    return BPJD_OK;
}

int bpjd_server_poll(bpjd_server* s, uint64_t req_id, double* eigvals, double* eigvecs, bpjd_stats* st) {
    bpjd::CtxScope cs_(s ? s->ctx : nullptr);
    if (!s) return bpjd::fail(BPJD_ERR_ARG, "NULL server");
    Request* r = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->all.find(req_id);
        if (it == s->all.end()) return bpjd::fail(BPJD_ERR_ARG, "unknown request id");
        r = it->second;
        if (r->state != Request::DONE) return BPJD_PENDING;
        s->all.erase(it);
    }
    if (eigvals && !r->eigvals.empty()) std::memcpy(eigvals, r->eigvals.data(), sizeof(double) * r->eigvals.size());
    if (eigvecs && !r->eigvecs.empty()) std::memcpy(eigvecs, r->eigvecs.data(), sizeof(double) * r->eigvecs.size());
    if (st) *st = r->stats;
    const int rc = r->rc;
    if (rc < 0) bpjd::set_error(r->err);
    delete r;
    return rc;
}

int bpjd_server_get_info(bpjd_server* s, bpjd_server_info* out) {
    bpjd::CtxScope cs_(s ? s->ctx : nullptr);
    if (!s || !out) return bpjd::fail(BPJD_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->info;
    out->queued = (uint32_t)s->queued.size();
    out->running = (uint32_t)s->running.size();
    out->bytes_in_use = s->in_use;
    return BPJD_OK;
}

void bpjd_server_destroy(bpjd_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_admit.notify_all();
    s->cv_step.notify_all();
    s->cv_reap.notify_all();
    s->cv_plan.notify_all();
    for (auto& t : s->plan_thr) t.join();
    s->admit_thr.join();
    s->step_thr.join();
    s->reap_thr.join();
    // solves still on the device are drained before their memory is freed
    for (auto& c : s->slot_ctx) (void)hipStreamSynchronize(c->stream);
    for (auto& kv : s->all) {
        Request* r = kv.second;
        if (r->run) bpjd::run_destroy(r->run);
        if (r->p) bpjd_problem_destroy(r->p);
        if (r->planned_p) bpjd_problem_destroy(r->planned_p);
        delete r;
    }
    for (auto& c : s->slot_ctx) {
        (void)hipStreamDestroy(c->stream);
        if (c->hbuf) (void)hipHostFree(c->hbuf);
    }
    if (s->arena.base) {
        if (s->arena_route == 1) s->ctx->alloc.free(s->arena.base, s->ctx->alloc.user);
        else (void)hipFree(s->arena.base);
    }
    delete s;
}

}  // extern "C"
