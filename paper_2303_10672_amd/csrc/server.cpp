// Request server: continuous batching of value-iteration solves on one GPU.
//
// Requests enter a queue with their arrival time.  Worker threads take them as
// soon as device memory and a worker are free:
//  * small scenario-A instances (both value tables fit in one workgroup's LDS) go
//    to the batch workers, which pack up to small_batch of them into one launch of
//    the batched kernel on their own stream; a request that arrives while a batch
//    runs joins the next batch of whichever batch worker frees first;
//  * everything else goes to the large workers, which run the ordinary sweep loop
//    (vi_solve) on their own streams, so large solves overlap with the batches.
// Admission: a large request is started only when its device bytes fit both the
// server budget and the free device memory; one that can never fit completes with
// PVI_E_BUSY.  The V table of a large request stays resident in HBM until its
// solve converges; if the request made the handle resident, its results then move
// to the handle's host memory and its device buffers are freed, so finished
// handles that the caller keeps never hold memory that waiting requests need.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>
#include <vector>

#include "families.h"
#include "mdp.h"

namespace {

using clk = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    pvi_mdp* mdp = nullptr;
    pvi_solve_opts opts{};
    std::vector<double> v0;
    clk::time_point t_submit;
    bool small = false;
    int64_t bytes = 0;
    int done = 0;
    pvi_status status = PVI_OK;
    pvi_result res{};
};

constexpr int kSmallMaxLds = 60 * 1024;

size_t small_lds_bytes(const pvi_mdp* p) {
    return sizeof(double) * (2 * (size_t)p->ns + 3 * (size_t)p->tab + p->a_r0.size());
}

// The batched kernel runs FIFO scenario A under the span rule; everything else
// takes the sweep loop.
bool is_small(const pvi_mdp* p, const pvi_solve_opts& o) {
    return p->family == PVI_FAMILY_LEADTIME && p->d.issuing == PVI_FIFO &&
           o.stop_rule == PVI_STOP_SPAN && o.v0 == nullptr && p->rad[0] <= 24 &&
           small_lds_bytes(p) <= kSmallMaxLds;
}

}  // namespace

struct pvi_server {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> small_q, large_q;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    std::vector<double> latency_ms;
    uint64_t next_ticket = 1;
    int64_t budget = 0, used = 0;
    int small_batch = 256;
    int device = 0;
    bool stop = false;
    std::vector<std::thread> workers;
};

namespace {

void finish(pvi_server* S, Request* r) {
    const double ms =
        std::chrono::duration<double, std::milli>(clk::now() - r->t_submit).count();
    r->res.wall_ms = ms;
    r->res.status = r->status;
    r->done = 1;
    S->latency_ms.push_back(ms);
}

void large_worker(pvi_server* S) {
    (void)hipSetDevice(S->device);
    hipStream_t stream;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) return;
    for (;;) {
        Request* r = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] {
                if (S->stop) return true;
                if (S->large_q.empty()) return false;
                Request* f = S->large_q.front();
                if (f->bytes > S->budget) return true;  // can never fit: complete as BUSY
                size_t fr = 0, tot = 0;
                if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = 0;
                return S->used + f->bytes <= S->budget &&
                       (f->mdp->dev.ready || (int64_t)fr > f->bytes + (64 << 20));
            });
            if (S->stop && S->large_q.empty()) break;
            if (S->large_q.empty()) continue;
            r = S->large_q.front();
            S->large_q.pop_front();
            if (r->bytes > S->budget) {
                r->status = PVI_E_BUSY;
                finish(S, r);
                S->cv_done.notify_all();
                continue;
            }
            S->used += r->bytes;
        }
        pvi_solve_opts o = r->opts;
        o.stream = stream;
        o.v0 = r->v0.empty() ? nullptr : r->v0.data();
        pvi_result res{};
        const bool fresh = !r->mdp->dev.ready;
        // direct launches: two workers solve at once on their own streams, and
        // captured graphs are kept to single-caller solves
        pvi_status st = pvi::solve_impl(r->mdp, &o, &res, false);
        // a handle this request made resident returns its HBM with the results in
        // host memory, so finished requests never block the admission of new ones
        if (fresh && (st == PVI_OK || st == PVI_E_NOT_CONVERGED)) {
            const pvi_status ps = pvi::park_results(r->mdp);
            if (ps != PVI_OK) st = ps;
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->used -= r->bytes;
            r->res = res;
            r->status = st;
            finish(S, r);
        }
        S->cv_done.notify_all();
        S->cv_work.notify_all();
    }
    (void)hipStreamDestroy(stream);
}

// Device arena of one batch worker: items, per-instance tables and outputs.
struct Arena {
    size_t bytes = 0;
    char* d = nullptr;
    char* h = nullptr;  // pinned staging copy
};

void small_worker(pvi_server* S) {
    (void)hipSetDevice(S->device);
    hipStream_t stream;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) return;
    Arena ar;
    // take the arena up front so the first batch does not pay for allocation
    {
        const size_t want = size_t(32) << 20;
        if (hipMalloc((void**)&ar.d, want) == hipSuccess &&
            hipHostMalloc((void**)&ar.h, want, hipHostMallocDefault) == hipSuccess) {
            ar.bytes = want;
        } else {
            if (ar.d) (void)hipFree(ar.d);
            if (ar.h) (void)hipHostFree(ar.h);
            ar = Arena{};
        }
    }
    for (;;) {
        std::vector<Request*> batch;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] { return S->stop || !S->small_q.empty(); });
            if (S->stop && S->small_q.empty()) break;
            while (!S->small_q.empty() && (int)batch.size() < S->small_batch) {
                batch.push_back(S->small_q.front());
                S->small_q.pop_front();
            }
        }
        // layout: items | per instance: tables, V, gap, policy, stats (8-byte aligned)
        const int n = (int)batch.size();
        size_t off = sizeof(pvi::BatchItem) * n;
        off = (off + 255) & ~size_t(255);
        std::vector<size_t> base(n);
        size_t lds = 0;
        int rmax = 1;
        for (int i = 0; i < n; ++i) {
            const pvi_mdp* p = batch[i]->mdp;
            base[i] = off;
            off += sizeof(double) * (3 * (size_t)p->tab + p->a_r0.size());
            off += sizeof(double) * (2 * (size_t)p->ns + 8) + sizeof(int32_t) * p->ns;
            off = (off + 15) & ~size_t(15);
            lds = std::max(lds, small_lds_bytes(p));
            rmax = std::max(rmax, p->rad[0]);
        }
        pvi_status st = PVI_OK;
        if (off > ar.bytes) {
            if (ar.d) (void)hipFree(ar.d);
            if (ar.h) (void)hipHostFree(ar.h);
            ar = Arena{};
            const size_t want = std::max(off, size_t(8) << 20);
            if (hipMalloc((void**)&ar.d, want) != hipSuccess ||
                hipHostMalloc((void**)&ar.h, want, hipHostMallocDefault) != hipSuccess) {
                st = PVI_E_NOMEM;
            } else {
                ar.bytes = want;
            }
        }
        if (st == PVI_OK) {
            auto* items = reinterpret_cast<pvi::BatchItem*>(ar.h);
            for (int i = 0; i < n; ++i) {
                const Request* r = batch[i];
                const pvi_mdp* p = r->mdp;
                char* hb = ar.h + base[i];
                char* db = ar.d + base[i];
                const size_t t = sizeof(double) * p->tab;
                std::memcpy(hb, p->a_pmf.data(), t);
                std::memcpy(hb + t, p->a_cdf.data(), t);
                std::memcpy(hb + 2 * t, p->a_tail.data(), t);
                std::memcpy(hb + 3 * t, p->a_r0.data(), sizeof(double) * p->a_r0.size());
                const size_t o_v = 3 * t + sizeof(double) * p->a_r0.size();
                const size_t o_gap = o_v + sizeof(double) * p->ns;
                const size_t o_st = o_gap + sizeof(double) * p->ns;
                const size_t o_pi = o_st + sizeof(double) * 8;
                pvi::BatchItem& it = items[i];
                it = pvi::BatchItem{};
                it.m = p->m;
                it.R = p->rad[0];
                it.dmax = p->dmax[0];
                it.tab = p->tab;
                it.xt = p->xt;
                it.ns = (int)p->ns;
                int nh = 1;
                for (int k = 0; k < p->L - 1; ++k) nh *= p->rad[0];
                it.nh = nh;
                int sh = 1;
                for (int k = 0; k < p->m - 1; ++k) sh *= p->rad[0];
                it.stride_h = sh;
                it.stride_a = sh * nh;
                it.max_sweeps = r->opts.max_sweeps > 0 ? r->opts.max_sweeps : r->opts.fixed_sweeps;
                it.fixed = r->opts.fixed_sweeps;
                it.fp32 = r->opts.precision != PVI_FP64;
                it.gamma = p->d.gamma;
                it.cvar = p->d.c_var[0];
                it.thr = r->opts.eps * (1.0 - p->d.gamma) / p->d.gamma;
                auto* dd = reinterpret_cast<double*>(db);
                it.pmf = dd;
                it.cdf = dd + p->tab;
                it.tail = dd + 2 * p->tab;
                it.r0 = dd + 3 * p->tab;
                it.v = reinterpret_cast<double*>(db + o_v);
                it.gap = reinterpret_cast<double*>(db + o_gap);
                it.stats = reinterpret_cast<double*>(db + o_st);
                it.pi = reinterpret_cast<int32_t*>(db + o_pi);
            }
            const auto t0 = clk::now();
            if (hipMemcpyAsync(ar.d, ar.h, off, hipMemcpyHostToDevice, stream) != hipSuccess ||
                pvi::launch_batch(reinterpret_cast<pvi::BatchItem*>(ar.d), n, lds, rmax,
                                  stream) != hipSuccess ||
                hipMemcpyAsync(ar.h, ar.d, off, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                hipStreamSynchronize(stream) != hipSuccess)
                st = PVI_E_DEVICE;
            const double dev_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
            if (st == PVI_OK) {
                for (int i = 0; i < n; ++i) {
                    Request* r = batch[i];
                    pvi_mdp* p = r->mdp;
                    const char* hb = ar.h + base[i];
                    const size_t t = sizeof(double) * p->tab;
                    const size_t o_v = 3 * t + sizeof(double) * p->a_r0.size();
                    const size_t o_gap = o_v + sizeof(double) * p->ns;
                    const size_t o_st = o_gap + sizeof(double) * p->ns;
                    const size_t o_pi = o_st + sizeof(double) * 8;
                    const double* stt = reinterpret_cast<const double*>(hb + o_st);
                    {
                        std::lock_guard<std::mutex> lk(p->mu);
                        p->h_v.assign(reinterpret_cast<const double*>(hb + o_v),
                                      reinterpret_cast<const double*>(hb + o_v) + p->ns);
                        p->h_gap.assign(reinterpret_cast<const double*>(hb + o_gap),
                                        reinterpret_cast<const double*>(hb + o_gap) + p->ns);
                        p->h_pi.assign(reinterpret_cast<const int32_t*>(hb + o_pi),
                                       reinterpret_cast<const int32_t*>(hb + o_pi) + p->ns);
                        p->have_result = 2;
                    }
                    pvi_result& res = r->res;
                    std::memset(&res, 0, sizeof(res));
                    res.sweeps_fp32 = (int32_t)stt[0];
                    res.sweeps_fp64 = (int32_t)stt[1];
                    res.final_span = stt[2];
                    res.dmax = stt[3];
                    res.dmin = stt[4];
                    res.threshold = r->opts.eps * (1.0 - p->d.gamma) / p->d.gamma;
                    res.backup_ms[1] = dev_ms;  // the batch launch this request ran in
                    const int64_t sw = res.sweeps_fp32 + res.sweeps_fp64 + 1;
                    res.logical_backups = p->logical_per_sweep * sw;
                    res.executed_terms = p->executed_per_sweep * sw;
                    r->status = stt[5] == 0.0 ? PVI_OK : PVI_E_NOT_CONVERGED;
                }
            }
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (Request* r : batch) {
                if (st != PVI_OK) r->status = st;
                finish(S, r);
            }
        }
        S->cv_done.notify_all();
    }
    if (ar.d) (void)hipFree(ar.d);
    if (ar.h) (void)hipHostFree(ar.h);
    (void)hipStreamDestroy(stream);
}

}  // namespace

using pvi::fail;

extern "C" {

pvi_status pvi_server_create(int64_t hbm_budget_bytes, int32_t small_batch, pvi_server** out) {
    if (!out) return fail(PVI_E_INVALID, "pvi_server_create: NULL argument");
    if (small_batch < 0 || small_batch > 4096)
        return fail(PVI_E_INVALID, "pvi_server_create: small_batch must be in 0..4096");
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0)
        return fail(PVI_E_DEVICE, "no HIP device available (this library has no CPU path)");
    auto* S = new pvi_server();
    (void)hipGetDevice(&S->device);
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        delete S;
        return fail(PVI_E_DEVICE, "hipMemGetInfo failed");
    }
    S->budget = hbm_budget_bytes > 0 ? hbm_budget_bytes : (int64_t)(0.8 * (double)fr);
    S->small_batch = small_batch > 0 ? small_batch : 256;
    for (int i = 0; i < 2; ++i) S->workers.emplace_back(small_worker, S);
    for (int i = 0; i < 2; ++i) S->workers.emplace_back(large_worker, S);
    *out = S;
    return PVI_OK;
}

pvi_status pvi_server_destroy(pvi_server* S) {
    if (!S) return PVI_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        // requests that have not started are cancelled
        for (Request* r : S->small_q) {
            r->status = PVI_E_CANCELLED;
            finish(S, r);
        }
        for (Request* r : S->large_q) {
            r->status = PVI_E_CANCELLED;
            finish(S, r);
        }
        S->small_q.clear();
        S->large_q.clear();
    }
    S->cv_work.notify_all();
    for (auto& t : S->workers) t.join();
    delete S;
    return PVI_OK;
}

pvi_status vi_batch_submit(pvi_server* S, pvi_mdp* const* mdps, const pvi_solve_opts* opts_in,
                           int32_t n, uint64_t* tickets) {
    if (!S || !mdps || !opts_in || !tickets || n < 0)
        return fail(PVI_E_INVALID, "vi_batch_submit: NULL argument");
    // older callers' shorter options struct: missing fields read as zero
    if (opts_in->struct_size < offsetof(pvi_solve_opts, stop_rule))
        return fail(PVI_E_INVALID, "vi_batch_submit: struct_size too small");
    pvi_solve_opts oc{};
    std::memcpy(&oc, opts_in, std::min<size_t>(opts_in->struct_size, sizeof(pvi_solve_opts)));
    oc.struct_size = sizeof(pvi_solve_opts);
    const pvi_solve_opts* opts = &oc;
    if (opts->stop_rule != PVI_STOP_SPAN && opts->stop_rule != PVI_STOP_SUPNORM &&
        opts->stop_rule != PVI_STOP_PERIODIC)
        return fail(PVI_E_INVALID, "vi_batch_submit: bad stop_rule");
    if (opts->checkpoint_path || opts->checkpoint_every != 0 || opts->resume != 0)
        return fail(PVI_E_INVALID, "vi_batch_submit: checkpoint files are not served; "
                                   "call vi_solve");
    for (int i = 0; i < n; ++i) {
        if (!mdps[i]) return fail(PVI_E_INVALID, "vi_batch_submit: NULL handle");
        if (!pvi::family_supported(mdps[i]))
            return fail(PVI_E_INVALID, "vi_batch_submit: " + pvi::family_support_msg(mdps[i]));
    }
    if (!(opts->eps > 0.0) || (opts->max_sweeps <= 0 && opts->fixed_sweeps <= 0))
        return fail(PVI_E_INVALID, "vi_batch_submit: bad options");
    const auto now = clk::now();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) return fail(PVI_E_CANCELLED, "vi_batch_submit: server is shutting down");
        for (int i = 0; i < n; ++i) {
            auto r = std::make_unique<Request>();
            r->ticket = S->next_ticket++;
            r->mdp = mdps[i];
            r->opts = *opts;
            r->opts.stream = nullptr;
            if (opts->v0) r->v0.assign(opts->v0, opts->v0 + mdps[i]->ns);
            r->t_submit = now;
            r->small = S->small_batch > 0 && is_small(mdps[i], *opts);
            r->bytes = r->small ? 0 : (int64_t)pvi::device_bytes(mdps[i]);
            tickets[i] = r->ticket;
            (r->small ? S->small_q : S->large_q).push_back(r.get());
            S->reqs[r->ticket] = std::move(r);
        }
    }
    S->cv_work.notify_all();
    return PVI_OK;
}

static pvi_status ticket_result(pvi_server* S, uint64_t ticket, pvi_result* res, bool* done) {
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(PVI_E_INVALID, "unknown ticket");
    Request* r = it->second.get();
    *done = r->done != 0;
    if (*done && res) *res = r->res;
    return PVI_OK;
}

pvi_status vi_poll(pvi_server* S, uint64_t ticket, pvi_result* res) {
    if (!S) return fail(PVI_E_INVALID, "vi_poll: NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    bool done = false;
    pvi_status st = ticket_result(S, ticket, res, &done);
    if (st != PVI_OK) return st;
    if (!done) return PVI_E_NOT_READY;
    return S->reqs[ticket]->status;
}

pvi_status vi_wait(pvi_server* S, uint64_t ticket, int64_t timeout_us, pvi_result* res) {
    if (!S) return fail(PVI_E_INVALID, "vi_wait: NULL server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(PVI_E_INVALID, "vi_wait: unknown ticket");
    Request* r = it->second.get();
    auto ready = [&] { return r->done != 0; };
    if (timeout_us < 0) {
        S->cv_done.wait(lk, ready);
    } else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
        return PVI_E_NOT_READY;
    }
    if (res) *res = r->res;
    return r->status;
}

pvi_status pvi_server_stats(pvi_server* S, double* p50, double* p99, int64_t* completed) {
    if (!S) return fail(PVI_E_INVALID, "pvi_server_stats: NULL server");
    std::vector<double> v;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        v = S->latency_ms;
    }
    if (completed) *completed = (int64_t)v.size();
    if (v.empty()) {
        if (p50) *p50 = 0.0;
        if (p99) *p99 = 0.0;
        return PVI_OK;
    }
    std::sort(v.begin(), v.end());
    auto q = [&](double f) {
        const double k = f * (v.size() - 1);
        const size_t lo = (size_t)k, hi = std::min(lo + 1, v.size() - 1);
        return v[lo] + (v[hi] - v[lo]) * (k - lo);
    };
    if (p50) *p50 = q(0.5);
    if (p99) *p99 = q(0.99);
    return PVI_OK;
}

}  // extern "C"
