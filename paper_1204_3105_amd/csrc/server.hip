// server.hip -- serving loop: continuous batching of independent solves.
//
// A scheduler thread owns two HIP streams (default priority).  Requests are
// admitted in arrival order while their device-memory estimate fits the
// budget (a request larger than the whole budget runs when nothing else is
// resident).  Admitted requests are planned on the planning stream while the
// previous batch evaluates on the evaluation stream; when the evaluation
// stream is idle, every planned request joins the next batch, whose phases
// (P2M, M2M, M2L, L2L, L2P + P2P) are each one launch over all of them
// (run_batch).  A finished batch's results are copied back, its plans
// destroyed and its memory returned to the budget.  Each request's numbers
// are the same as a standalone fmm_plan + fmm_eval: an item's arithmetic
// depends only on its own plan's data.
#include <string.h>

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
    double *d_pts = nullptr, *d_tgt = nullptr, *d_u = nullptr;
    size_t pts_bytes = 0, tgt_bytes = 0, u_bytes = 0;
    int64_t reserved = 0;
    int p = 0, lmax = 0;
};

struct Server {
    fmm_server_options opt{};
    std::thread th;
    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::deque<Req *> queue;
    std::map<uint64_t, Req *> all;
    std::vector<Req *> planned, running;
    uint64_t next_ticket = 1;
    int64_t used = 0;
    int admitted = 0;
    bool stop = false;
    hipStream_t s_plan = nullptr, s_eval = nullptr, s_near = nullptr;
    hipEvent_t done_ev = nullptr;
    hipEvent_t bev[7] = {};   // run_batch stage, fork and near-field events
    EvalJob *jobs = nullptr;
    size_t jobs_cap = 0;
    int device = 0;
};

static int64_t estimate_bytes(const Req &r)
{
    const int64_t pts = r.n_src + (r.same ? 0 : r.n_tgt);
    return (int64_t)400 * pts + ((int64_t)32 << 20);
}

static void free_inputs(Req *r)
{
    dev_free(r->d_pts, r->pts_bytes);
    if (r->d_tgt) dev_free(r->d_tgt, r->tgt_bytes);
    dev_free(r->d_u, r->u_bytes);
    r->d_pts = r->d_tgt = r->d_u = nullptr;
}

// Plan one request on the planning stream.  Returns false on failure (the
// request is then finished with its error status).
static bool plan_request(Server &S, Req *r)
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
        r->status = FMM_E_NOMEM;
        return false;
    }
    if (r->n_src) {
        hipMemcpyAsync(r->d_pts, r->src.data(), 16 * r->n_src, hipMemcpyHostToDevice, S.s_plan);
        hipMemcpyAsync(r->d_u, r->u.data(), 8 * r->n_src, hipMemcpyHostToDevice, S.s_plan);
    }
    if (!r->same && r->n_tgt)
        hipMemcpyAsync(r->d_tgt, r->tgt.data(), 16 * r->n_tgt, hipMemcpyHostToDevice, S.s_plan);
    fmm_options o;
    fmm_options_default(&o);
    o.leaf_size = S.opt.leaf_size > 0 ? S.opt.leaf_size : 64;
    o.precision = r->precision;
    o.device_pointers = 1;
    o.stream = (void *)S.s_plan;
    const double *tgt = r->same ? r->d_pts : r->d_tgt;
    fmm_status st = fmm_plan((fmm_tiling)r->tiling, r->d_pts, r->n_src, tgt, r->n_tgt, r->eps, &o,
                             &r->plan);
    hipStreamSynchronize(S.s_plan);
    if (st != FMM_OK) {
        r->status = st;
        return false;
    }
    // Sizes straight from the plan (fmm_plan_info_get would also count the
    // interaction pairs, which the scheduler does not need).
    const Plan *P = (const Plan *)r->plan;
    r->reserved = plan_device_bytes(P) + (int64_t)(r->pts_bytes + r->tgt_bytes + r->u_bytes);
    r->p = P->p;
    r->lmax = P->geo.L;
    return true;
}

static void finish(Server &S, Req *r, bool ok)
{
    if (r->plan) {
        fmm_plan_destroy(r->plan);
        r->plan = nullptr;
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

static void launch_batch(Server &S, std::vector<Req *> &batch)
{
    const int n = (int)batch.size();
    if ((size_t)n > S.jobs_cap) {
        if (S.jobs) dev_free(S.jobs, S.jobs_cap * sizeof(EvalJob));
        int err = 0;
        S.jobs_cap = (size_t)std::max(n, 64);
        S.jobs = (EvalJob *)dev_alloc(S.jobs_cap * sizeof(EvalJob), &err);
    }
    std::vector<Plan *> plans;
    std::vector<Req *> work;
    for (Req *r : batch) {
        Plan *P = (Plan *)r->plan;
        r->t_start = now_s();
        if (P->n_tgt == 0) continue;
        if (P->n_src == 0) {
            hipMemsetAsync(P->phi_int, 0, sizeof(double) * 2 * P->n_tgt, S.s_eval);
            continue;
        }
        const int i = (int)plans.size();
        hipMemcpyAsync(S.jobs + i, P->job_dev, sizeof(EvalJob), hipMemcpyDeviceToDevice, S.s_eval);
        plans.push_back(P);
        work.push_back(r);
    }
    for (size_t i = 0; i < plans.size(); ++i) {
        EvalJob J = make_job(*plans[i]);
        batch_gather_u(S.jobs, J, work[i]->d_u, S.s_eval);
    }
    if (!plans.empty())
        run_batch(plans.data(), (int)plans.size(), S.jobs, nullptr, S.s_eval, S.s_near, S.bev);
    hipEventRecord(S.done_ev, S.s_eval);
}

static void complete_batch(Server &S, std::vector<Req *> &batch)
{
    for (Req *r : batch) {
        Plan *P = (Plan *)r->plan;
        r->phi.resize(2 * (size_t)r->n_tgt);
        bool ok = true;
        if (r->n_tgt)
            ok = hipMemcpy(r->phi.data(), P->phi_int, sizeof(double) * 2 * r->n_tgt,
                           hipMemcpyDeviceToHost) == hipSuccess;
        finish(S, r, ok);
    }
    S.cv_done.notify_all();
}

// Whether the event has passed; a "not ready" answer is not kept as the
// thread's last error (plan building checks that).
static bool done_query(hipEvent_t ev)
{
    const hipError_t e = hipEventQuery(ev);
    if (e == hipErrorNotReady && hipPeekAtLastError() == hipErrorNotReady) (void)hipGetLastError();
    return e == hipSuccess;
}

static void scheduler(Server *Sp)
{
    Server &S = *Sp;
    hipSetDevice(S.device);
    for (;;) {
        bool progress = false;
        // 1. completion of the running batch
        if (!S.running.empty() && done_query(S.done_ev)) {
            complete_batch(S, S.running);
            S.running.clear();
            progress = true;
        }
        // 2. admission and planning
        for (;;) {
            Req *r = nullptr;
            {
                std::lock_guard<std::mutex> lk(S.mu);
                if (S.queue.empty() || S.admitted >= S.opt.max_inflight) break;
                Req *h = S.queue.front();
                const int64_t est = estimate_bytes(*h);
                if (S.admitted > 0 && S.used + est > S.opt.hbm_budget_bytes) break;
                S.queue.pop_front();
                S.used += est;
                S.admitted++;
                h->reserved = est;
                h->t_admit = now_s();
                r = h;
            }
            const int64_t est = r->reserved;
            const bool ok = plan_request(S, r);
            {
                std::lock_guard<std::mutex> lk(S.mu);
                if (ok) S.used += r->reserved - est;
                else r->reserved = est;
            }
            if (ok)
                S.planned.push_back(r);
            else
                finish(S, r, false);
            progress = true;
            // Start evaluating as soon as the GPU is free.
            if (S.running.empty()) break;
            if (done_query(S.done_ev)) break;
        }
        // 3. launch the next batch
        if (S.running.empty() && !S.planned.empty()) {
            S.running.swap(S.planned);
            launch_batch(S, S.running);
            progress = true;
        }
        if (!progress) {
            std::unique_lock<std::mutex> lk(S.mu);
            if (S.stop && S.queue.empty() && S.running.empty() && S.planned.empty()) break;
            S.cv.wait_for(lk, std::chrono::microseconds(S.running.empty() ? 2000 : 50));
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
    hipGetDevice(&S->device);
    if (hipStreamCreateWithFlags(&S->s_plan, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&S->s_eval, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&S->s_near, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&S->done_ev, hipEventDisableTiming) != hipSuccess) {
        set_error("stream or event creation failed");
        delete S;
        return FMM_E_DEVICE;
    }
    for (auto &e : S->bev) {
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            set_error("event creation failed");
            delete S;
            return FMM_E_DEVICE;
        }
    }
    S->th = std::thread(scheduler, S);
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
    S->cv.notify_all();
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
        S->cv.notify_all();
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
    S->cv.notify_all();
    if (S->th.joinable()) S->th.join();
    for (auto &kv : S->all) delete kv.second;
    if (S->jobs) dev_free(S->jobs, S->jobs_cap * sizeof(EvalJob));
    hipEventDestroy(S->done_ev);
    for (auto &e : S->bev) hipEventDestroy(e);
    hipStreamDestroy(S->s_plan);
    hipStreamDestroy(S->s_eval);
    hipStreamDestroy(S->s_near);
    delete S;
    return FMM_OK;
}

}  // extern "C"
