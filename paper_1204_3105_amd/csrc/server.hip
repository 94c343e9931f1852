// server.hip -- serving loop: continuous batching of independent solves.
//
// Two host threads share a request queue.  The planner admits requests in
// arrival order while their device-memory estimate fits the budget (a
// request larger than the whole budget runs when nothing else is resident)
// and plans each on the planning stream without waiting for it: an event
// recorded behind the plan marks it ready.  The scheduler keeps up to
// kEvalSlots batches in flight, each on an evaluation stream of its own:
// whenever a slot is free, every planned request joins a new batch there,
// whose phases (P2M, M2M, M2L, L2L, P2P, L2P) are each one launch over all of
// them (run_batch, near field on the batch's stream), after the stream has
// waited for their plans' events.  So requests planned while a batch runs
// start at once on the other slot and overlap it on the device; a small
// request can finish before a large one submitted earlier.  A finished
// batch's results are copied back, its plans destroyed and its memory
// returned to the budget.  Each request's numbers are the same as a
// standalone fmm_plan + fmm_eval: an item's arithmetic depends only on its
// own plan's data.  Streams: one planning and kEvalSlots evaluation streams,
// within the four hardware queues a process gets.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "eval.h"

namespace fmm {

static double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr int kEvalSlots = 2;

struct Req {
    uint64_t ticket = 0;
    int tiling = 0, precision = 0;
    double eps = 0;
    int64_t n_src = 0, n_tgt = 0;
    bool same = false;
    std::vector<double> src, tgt, u, phi;
    double t_submit = 0, t_admit = 0, t_start = 0, t_end = 0;
    bool done = false;
    fmm_status status = FMM_OK;
    fmm_plan_t plan = nullptr;
    hipEvent_t ready = nullptr;   // recorded behind the plan on the planning stream
    double *d_pts = nullptr, *d_tgt = nullptr, *d_u = nullptr;
    size_t pts_bytes = 0, tgt_bytes = 0, u_bytes = 0;
    int64_t reserved = 0;
    int p = 0, lmax = 0;
};

struct Slot {
    std::vector<Req *> reqs;
    hipStream_t s = nullptr;
    hipEvent_t done = nullptr;
    hipEvent_t bev[7] = {};   // run_batch stage, fork and near-field events
    EvalJob *jobs = nullptr;
    size_t jobs_cap = 0;
    bool busy = false;
};

struct Server {
    fmm_server_options opt{};
    std::thread th_sched, th_plan;
    std::mutex mu;
    std::condition_variable cv_sched, cv_plan, cv_done;
    std::deque<Req *> queue;
    std::map<uint64_t, Req *> all;
    std::vector<Req *> planned;
    uint64_t next_ticket = 1;
    int64_t used = 0;
    int64_t budget = 0;
    int admitted = 0;
    int planning = 0;   // requests admitted and being planned
    bool stop = false;
    hipStream_t s_plan = nullptr;
    Slot slot[kEvalSlots];
    int device = 0;
};

static int64_t estimate_bytes(const Server &S, const Req &r)
{
    return plan_bytes_estimate(r.tiling, r.n_src, r.n_tgt, r.same, r.eps, r.precision,
                               S.opt.leaf_size > 0 ? S.opt.leaf_size : 64) +
           (int64_t)24 * (r.n_src + (r.same ? 0 : r.n_tgt));
}

static void free_inputs(Req *r)
{
    if (r->d_pts) dev_free(r->d_pts, r->pts_bytes);
    if (r->d_tgt) dev_free(r->d_tgt, r->tgt_bytes);
    if (r->d_u) dev_free(r->d_u, r->u_bytes);
    r->d_pts = r->d_tgt = r->d_u = nullptr;
}

// Plan one request on the planning stream, without waiting for the plan's
// last kernels (r->ready marks them).  Returns the status.
static fmm_status plan_request(Server &S, Req *r)
{
    int err = 0;
    r->pts_bytes = (size_t)std::max<int64_t>(r->n_src, 1) * 16;
    r->u_bytes = (size_t)std::max<int64_t>(r->n_src, 1) * 8;
    r->d_pts = (double *)dev_alloc(r->pts_bytes, &err);
    r->d_u = (double *)dev_alloc(r->u_bytes, &err);
    if (!r->same) {
        r->tgt_bytes = (size_t)std::max<int64_t>(r->n_tgt, 1) * 16;
        r->d_tgt = (double *)dev_alloc(r->tgt_bytes, &err);
    }
    if (err) {
        free_inputs(r);
        return FMM_E_NOMEM;
    }
    if ((r->n_src && (hipMemcpyAsync(r->d_pts, r->src.data(), 16 * r->n_src, hipMemcpyHostToDevice,
                                     S.s_plan) != hipSuccess ||
                      hipMemcpyAsync(r->d_u, r->u.data(), 8 * r->n_src, hipMemcpyHostToDevice, S.s_plan) !=
                          hipSuccess)) ||
        (!r->same && r->n_tgt &&
         hipMemcpyAsync(r->d_tgt, r->tgt.data(), 16 * r->n_tgt, hipMemcpyHostToDevice, S.s_plan) != hipSuccess)) {
        (void)hipGetLastError();
        hipStreamSynchronize(S.s_plan);
        free_inputs(r);
        return FMM_E_DEVICE;
    }
    fmm_options o;
    fmm_options_default(&o);
    o.leaf_size = S.opt.leaf_size > 0 ? S.opt.leaf_size : 64;
    o.precision = r->precision;
    o.device_pointers = 1;
    o.stream = (void *)S.s_plan;
    o.near_stream = 1;   // the batch runs the near field on its own stream
    const double *tgt = r->same ? r->d_pts : r->d_tgt;
    fmm_status st = fmm_plan((fmm_tiling)r->tiling, r->d_pts, r->n_src, tgt, r->n_tgt, r->eps, &o,
                             &r->plan);
    if (st == FMM_OK && (hipEventCreateWithFlags(&r->ready, hipEventDisableTiming) != hipSuccess ||
                         hipEventRecord(r->ready, S.s_plan) != hipSuccess)) {
        (void)hipGetLastError();
        st = FMM_E_DEVICE;
    }
    if (st != FMM_OK) {
        if (r->plan) {
            fmm_plan_destroy(r->plan);
            r->plan = nullptr;
        }
        if (r->ready) {
            hipEventDestroy(r->ready);
            r->ready = nullptr;
        }
        hipStreamSynchronize(S.s_plan);   // the input copies are done before their memory goes back
        free_inputs(r);
        return st;
    }
    // Sizes straight from the plan (fmm_plan_info_get would also count the
    // interaction pairs, which the scheduler does not need).
    const Plan *P = (const Plan *)r->plan;
    r->reserved = plan_device_bytes(P) + (int64_t)(r->pts_bytes + r->tgt_bytes + r->u_bytes);
    r->p = P->p;
    r->lmax = P->geo.L;
    return FMM_OK;
}

// Release a request's device resources and publish its result; the caller
// has seen all of its device work finish.
static void finish(Server &S, Req *r, bool ok)
{
    if (r->plan) {
        fmm_plan_destroy(r->plan);
        r->plan = nullptr;
    }
    if (r->ready) {
        hipEventDestroy(r->ready);
        r->ready = nullptr;
    }
    free_inputs(r);
    if (!ok && r->status == FMM_OK) r->status = FMM_E_DEVICE;
    r->t_end = now_s();
    std::lock_guard<std::mutex> lk(S.mu);
    S.used -= r->reserved;
    S.admitted--;
    r->done = true;
    // release input copies early
    std::vector<double>().swap(r->src);
    std::vector<double>().swap(r->tgt);
    std::vector<double>().swap(r->u);
}

// Enqueue a batch on a slot's stream.  Returns false if the batch could not
// be started (its requests are then finished with FMM_E_NOMEM or
// FMM_E_DEVICE after the stream has drained).
static bool launch_batch(Server &S, Slot &L)
{
    const int n = (int)L.reqs.size();
    if ((size_t)n > L.jobs_cap) {
        if (L.jobs) dev_free(L.jobs, L.jobs_cap * sizeof(EvalJob));
        int err = 0;
        L.jobs_cap = (size_t)std::max(n, 64);
        L.jobs = (EvalJob *)dev_alloc(L.jobs_cap * sizeof(EvalJob), &err);
        if (err || !L.jobs) {
            L.jobs = nullptr;
            L.jobs_cap = 0;
            for (Req *r : L.reqs) r->status = FMM_E_NOMEM;
            return false;
        }
    }
    std::vector<Plan *> plans;
    std::vector<Req *> work;
    bool ok = true;
    for (Req *r : L.reqs) {
        Plan *P = (Plan *)r->plan;
        r->t_start = now_s();
        ok = ok && hipStreamWaitEvent(L.s, r->ready, 0) == hipSuccess;
        if (P->n_tgt == 0) continue;
        if (P->n_src == 0) {
            ok = ok && hipMemsetAsync(P->phi_int, 0, sizeof(double) * 2 * P->n_tgt, L.s) == hipSuccess;
            continue;
        }
        const int i = (int)plans.size();
        ok = ok && hipMemcpyAsync(L.jobs + i, P->job_dev, sizeof(EvalJob), hipMemcpyDeviceToDevice, L.s) ==
                       hipSuccess;
        plans.push_back(P);
        work.push_back(r);
    }
    for (size_t i = 0; i < plans.size(); ++i) {
        EvalJob J = make_job(*plans[i]);
        batch_gather_u(L.jobs, J, work[i]->d_u, L.s);
    }
    if (!plans.empty()) run_batch(plans.data(), (int)plans.size(), L.jobs, nullptr, L.s, L.s, L.bev);
    ok = ok && hipGetLastError() == hipSuccess;
    ok = ok && hipEventRecord(L.done, L.s) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        hipStreamSynchronize(L.s);
        for (Req *r : L.reqs) r->status = FMM_E_DEVICE;
    }
    return ok;
}

static void complete_batch(Server &S, Slot &L, bool launched)
{
    for (Req *r : L.reqs) {
        bool ok = launched;
        if (ok) {
            Plan *P = (Plan *)r->plan;
            r->phi.resize(2 * (size_t)r->n_tgt);
            if (r->n_tgt)
                ok = hipMemcpy(r->phi.data(), P->phi_int, sizeof(double) * 2 * r->n_tgt,
                               hipMemcpyDeviceToHost) == hipSuccess;
        }
        finish(S, r, ok);
    }
    L.reqs.clear();
    L.busy = false;
    S.cv_done.notify_all();
    S.cv_plan.notify_all();
}

// Whether the event has passed; a "not ready" answer is not kept as the
// thread's last error (plan building checks that).
static bool done_query(hipEvent_t ev)
{
    const hipError_t e = hipEventQuery(ev);
    if (e == hipErrorNotReady && hipPeekAtLastError() == hipErrorNotReady) (void)hipGetLastError();
    return e == hipSuccess;
}

// Admission and planning.
static void planner(Server *Sp)
{
    Server &S = *Sp;
    hipSetDevice(S.device);
    for (;;) {
        Req *r = nullptr;
        int64_t est = 0;
        {
            std::unique_lock<std::mutex> lk(S.mu);
            for (;;) {
                if (S.stop && S.queue.empty()) return;
                if (!S.queue.empty() && S.admitted < S.opt.max_inflight) {
                    Req *h = S.queue.front();
                    est = estimate_bytes(S, *h);
                    if (S.admitted == 0 || S.used + est <= S.budget) {
                        S.queue.pop_front();
                        S.used += est;
                        S.admitted++;
                        S.planning++;
                        if (h->t_admit == 0) h->t_admit = now_s();
                        r = h;
                        break;
                    }
                }
                S.cv_plan.wait_for(lk, std::chrono::milliseconds(2));
            }
        }
        const fmm_status st = plan_request(S, r);
        bool retry = false;
        {
            std::lock_guard<std::mutex> lk(S.mu);
            S.planning--;
            if (st == FMM_OK) {
                S.used += r->reserved - est;
                S.planned.push_back(r);
            } else if (st == FMM_E_NOMEM && S.admitted > 1) {
                // Memory is held by other resident requests: queue again at
                // the front and wait until one of them finishes.
                S.used -= est;
                S.admitted--;
                S.queue.push_front(r);
                retry = true;
            } else {
                r->reserved = est;
                r->status = st;
            }
        }
        if (st != FMM_OK && !retry) finish(S, r, false);
        S.cv_sched.notify_all();
        if (retry) {
            std::unique_lock<std::mutex> lk(S.mu);
            const int before = S.admitted;
            S.cv_done.wait_for(lk, std::chrono::milliseconds(50), [&] { return S.admitted < before || S.stop; });
        }
    }
}

// Batch launches and completions.
static void scheduler(Server *Sp)
{
    Server &S = *Sp;
    hipSetDevice(S.device);
    for (;;) {
        bool progress = false;
        for (Slot &L : S.slot)
            if (L.busy && done_query(L.done)) {
                complete_batch(S, L, true);
                progress = true;
            }
        for (Slot &L : S.slot) {
            if (L.busy) continue;
            {
                std::lock_guard<std::mutex> lk(S.mu);
                if (S.planned.empty()) break;
                L.reqs.swap(S.planned);
            }
            L.busy = true;
            if (!launch_batch(S, L)) complete_batch(S, L, false);
            progress = true;
        }
        if (!progress) {
            bool any_busy = false;
            for (Slot &L : S.slot) any_busy = any_busy || L.busy;
            std::unique_lock<std::mutex> lk(S.mu);
            if (S.stop && S.queue.empty() && S.planned.empty() && S.planning == 0 && !any_busy) break;
            S.cv_sched.wait_for(lk, std::chrono::microseconds(any_busy ? 50 : 2000));
        }
    }
}

}  // namespace fmm

using namespace fmm;

extern "C" {

fmm_status fmm_server_create(const fmm_server_options *opt, fmm_server_t *out)
{
    if (!out) {
        set_error("null output pointer");
        return FMM_E_INVALID;
    }
    *out = nullptr;
    if (!opt || opt->struct_size != sizeof(fmm_server_options) || opt->hbm_budget_bytes <= 0 ||
        opt->max_inflight <= 0) {
        set_error("bad server options");
        return FMM_E_INVALID;
    }
    Server *S = new Server();
    S->opt = *opt;
    S->budget = opt->hbm_budget_bytes;
    hipGetDevice(&S->device);
    {
        // The budget never exceeds 90% of what the device has free now.
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess && fr > 0)
            S->budget = std::min<int64_t>(S->budget, (int64_t)(0.9 * (double)fr));
        else
            (void)hipGetLastError();
    }
    bool ok = hipStreamCreateWithFlags(&S->s_plan, hipStreamNonBlocking) == hipSuccess;
    for (Slot &L : S->slot) {
        ok = ok && hipStreamCreateWithFlags(&L.s, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&L.done, hipEventDisableTiming) == hipSuccess;
        for (auto &e : L.bev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        set_error("stream or event creation failed");
        for (Slot &L : S->slot) {
            if (L.s) hipStreamDestroy(L.s);
            if (L.done) hipEventDestroy(L.done);
            for (auto &e : L.bev)
                if (e) hipEventDestroy(e);
        }
        if (S->s_plan) hipStreamDestroy(S->s_plan);
        delete S;
        return FMM_E_DEVICE;
    }
    S->th_plan = std::thread(planner, S);
    S->th_sched = std::thread(scheduler, S);
    *out = (fmm_server_t)S;
    return FMM_OK;
}

fmm_status fmm_submit(fmm_server_t s, const fmm_request *req, uint64_t *ticket)
{
    Server *S = (Server *)s;
    if (!S || !req || !ticket) {
        set_error("null argument");
        return FMM_E_INVALID;
    }
    if (req->tiling < 0 || req->tiling > 2 || req->n_src < 0 || req->n_tgt < 0 ||
        (req->n_src > 0 && (!req->src || !req->u)) || (req->tgt && req->n_tgt > 0 && !req->tgt) ||
        (!req->tgt && req->n_tgt != req->n_src) || !(req->eps > 0.0 && req->eps < 0.5) ||
        req->precision < 0 || req->precision > 2) {
        set_error("invalid request");
        return FMM_E_INVALID;
    }
    Req *r = new Req();
    r->tiling = req->tiling;
    r->precision = req->precision;
    r->eps = req->eps;
    r->n_src = req->n_src;
    r->n_tgt = req->n_tgt;
    r->same = req->tgt == nullptr;
    r->src.assign(req->src, req->src + 2 * req->n_src);
    if (!r->same) r->tgt.assign(req->tgt, req->tgt + 2 * req->n_tgt);
    r->u.assign(req->u, req->u + req->n_src);
    r->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        r->ticket = S->next_ticket++;
        S->all[r->ticket] = r;
        S->queue.push_back(r);
    }
    S->cv_plan.notify_all();
    *ticket = r->ticket;
    return FMM_OK;
}

fmm_status fmm_poll(fmm_server_t s, uint64_t ticket, double *phi, fmm_result *res)
{
    Server *S = (Server *)s;
    if (!S) {
        set_error("null server");
        return FMM_E_INVALID;
    }
    Req *r = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->all.find(ticket);
        if (it == S->all.end()) {
            set_error("unknown ticket");
            return FMM_E_INVALID;
        }
        if (!it->second->done) return FMM_E_BUSY;
        r = it->second;
        S->all.erase(it);
    }
    if (phi && r->status == FMM_OK && r->n_tgt)
        memcpy(phi, r->phi.data(), sizeof(double) * 2 * r->n_tgt);
    if (res) {
        res->status = r->status;
        res->p = r->p;
        res->lmax = r->lmax;
        res->t_submit = r->t_submit;
        res->t_admit = r->t_admit;
        res->t_start = r->t_start;
        res->t_end = r->t_end;
    }
    fmm_status st = r->status;
    delete r;
    return st == FMM_OK ? FMM_OK : st;
}

fmm_status fmm_server_drain(fmm_server_t s)
{
    Server *S = (Server *)s;
    if (!S) return FMM_E_INVALID;
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        bool busy = !S->queue.empty() || S->admitted > 0;
        if (!busy) return FMM_OK;
        S->cv_plan.notify_all();
        S->cv_sched.notify_all();
        S->cv_done.wait_for(lk, std::chrono::milliseconds(1));
    }
}

fmm_status fmm_server_destroy(fmm_server_t s)
{
    Server *S = (Server *)s;
    if (!S) return FMM_E_INVALID;
    fmm_server_drain(s);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_plan.notify_all();
    S->cv_sched.notify_all();
    if (S->th_plan.joinable()) S->th_plan.join();
    if (S->th_sched.joinable()) S->th_sched.join();
    for (auto &kv : S->all) delete kv.second;
    for (Slot &L : S->slot) {
        if (L.jobs) dev_free(L.jobs, L.jobs_cap * sizeof(EvalJob));
        hipEventDestroy(L.done);
        for (auto &e : L.bev) hipEventDestroy(e);
        hipStreamDestroy(L.s);
    }
    hipStreamDestroy(S->s_plan);
    delete S;
    return FMM_OK;
}

}  // extern "C"
