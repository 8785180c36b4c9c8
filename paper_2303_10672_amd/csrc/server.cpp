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
#include <atomic>
#include <chrono>
#include <cstddef>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

#include "families.h"
#include "mdp.h"
#include "server_core.h"
#include "slot_layout.h"
#include "slots.h"

namespace {

using clk = std::chrono::steady_clock;
using pvi::srv::Job;

struct Request : Job {
    pvi_mdp* mdp = nullptr;
    pvi_solve_opts opts{};
    std::vector<double> v0;
    pvi_result res{};
    std::atomic<int> sweeps{0};  // large requests: sweeps completed so far
};

constexpr int kSmallMaxLds = 60 * 1024;

size_t small_lds_bytes(const pvi_mdp* p) {
    return sizeof(double) * (2 * (size_t)p->ns + 3 * (size_t)p->tab + p->a_r0.size());
}

// The slot kernel runs FIFO scenario A under the span rule; everything else takes the
// sweep loop.
size_t slot_need(const pvi_mdp* p);

bool is_small(const pvi_mdp* p, const pvi_solve_opts& o) {
    return p->family == PVI_FAMILY_LEADTIME && p->d.issuing == PVI_FIFO &&
           o.stop_rule == PVI_STOP_SPAN && o.v0 == nullptr && p->rad[0] <= pvi::kSlotRmax &&
           small_lds_bytes(p) <= kSmallMaxLds && slot_need(p) <= (size_t(96) << 10);
}

}  // namespace

namespace {
struct HipSlotOps;
}  // namespace

struct pvi_server {
    std::unique_ptr<pvi::srv::Core> core;
    std::unique_ptr<HipSlotOps> slots;  // the small-instance slot kernel (null: none)
    int small_batch = 256;
    int device = 0;
    std::vector<std::thread> workers;
};

namespace {

void large_worker(pvi_server* S, int w) {
    (void)hipSetDevice(S->device);
    hipStream_t stream = nullptr;
    const bool have_stream = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess;
    auto free_bytes = [] {
        size_t fr = 0, tot = 0;
        return hipMemGetInfo(&fr, &tot) == hipSuccess ? (int64_t)fr : (int64_t)0;
    };
    for (;;) {
        Job* j = S->core->next_large(w, free_bytes, PVI_E_BUSY);
        if (!j) break;
        auto* r = static_cast<Request*>(j);
        pvi_status st = PVI_E_DEVICE;
        if (have_stream) {
            pvi_solve_opts o = r->opts;
            o.stream = stream;
            o.v0 = r->v0.empty() ? nullptr : r->v0.data();
            const bool fresh = !r->mdp->dev.ready;
            // direct launches: two workers solve at once on their own streams, and
            // captured graphs are kept to single-caller solves
            st = pvi::solve_impl(r->mdp, &o, &r->res, false, &r->sweeps);
            // a handle this request made resident returns its HBM with the results
            // in host memory, so finished requests never block the admission of
            // new ones
            if (fresh && (st == PVI_OK || st == PVI_E_NOT_CONVERGED)) {
                const pvi_status ps = pvi::park_results(r->mdp);
                if (ps != PVI_OK) st = ps;
            }
        }
        r->res.status = st;
        S->core->complete(r, st);
    }
    if (have_stream) (void)hipStreamDestroy(stream);
}

// Device side of the slot feeder: the slot table, one request arena per slot and the
// launches of the slot kernel, all in one block of coherent pinned host memory that
// the kernel reads and writes directly (the host never copies through the device).
// Per slot the arena holds the request's tables (P, F, G, reward), then its results
// (V, Q gap, 8 statistics, policy).
constexpr size_t kSlotArena = size_t(96) << 10;

size_t slot_need(const pvi_mdp* p) {
    return sizeof(double) * (3 * (size_t)p->tab + p->a_r0.size() + 2 * (size_t)p->ns + 8) +
           sizeof(int32_t) * (size_t)p->ns;
}

struct HipSlotOps : pvi::srv::SlotOps {
    int nslots = 0;
    int threads = 256;      // threads per slot work group
    size_t lds = 0;
    char* host = nullptr;   // the block (host address)
    char* dev = nullptr;    // the same block (device address)
    pvi::SlotHeader* hdr = nullptr;
    pvi::SlotSync* sync = nullptr;
    pvi::BatchItem* items = nullptr;
    size_t arena0 = 0;      // offset of slot 0's arena
    hipStream_t stream = nullptr;
    hipEvent_t done_ev = nullptr;
    bool launched = false;

    template <class T>
    T* dptr(T* h) const {
        return reinterpret_cast<T*>(dev + (reinterpret_cast<char*>(h) - host));
    }
    char* arena(int k) const { return host + arena0 + (size_t)k * kSlotArena; }

    bool init(int n) {
        nslots = n;
        lds = kSmallMaxLds;
        const size_t items_off = sizeof(pvi::SlotHeader) + sizeof(pvi::SlotSync) * (size_t)n;
        arena0 = (items_off + sizeof(pvi::BatchItem) * (size_t)n + 255) & ~size_t(255);
        const size_t bytes = arena0 + kSlotArena * (size_t)n;
        if (hipHostMalloc((void**)&host, bytes, hipHostMallocCoherent) != hipSuccess) {
            host = nullptr;
            return false;
        }
        std::memset(host, 0, bytes);
        void* d = nullptr;
        if (hipHostGetDevicePointer(&d, host, 0) != hipSuccess ||
            hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&done_ev, hipEventDisableTiming) != hipSuccess)
            return false;
        dev = static_cast<char*>(d);
        hdr = reinterpret_cast<pvi::SlotHeader*>(host);
        sync = reinterpret_cast<pvi::SlotSync*>(host + sizeof(pvi::SlotHeader));
        items = reinterpret_cast<pvi::BatchItem*>(host + items_off);
        return true;
    }
    ~HipSlotOps() override {
        if (launched) (void)hipEventSynchronize(done_ev);
        if (done_ev) (void)hipEventDestroy(done_ev);
        if (stream) (void)hipStreamDestroy(stream);
        if (host) (void)hipHostFree(host);
    }

    void prepare(int k, pvi::srv::Job* j) override {
        const auto* r = static_cast<Request*>(j);
        const pvi_mdp* p = r->mdp;
        char* hb = arena(k);
        const size_t t = sizeof(double) * p->tab;
        std::memcpy(hb, p->a_pmf.data(), t);
        std::memcpy(hb + t, p->a_cdf.data(), t);
        std::memcpy(hb + 2 * t, p->a_tail.data(), t);
        std::memcpy(hb + 3 * t, p->a_r0.data(), sizeof(double) * p->a_r0.size());
        const size_t o_v = 3 * t + sizeof(double) * p->a_r0.size();
        const size_t o_gap = o_v + sizeof(double) * p->ns;
        const size_t o_st = o_gap + sizeof(double) * p->ns;
        const size_t o_pi = o_st + sizeof(double) * 8;
        pvi::BatchItem it{};
        it.m = p->m;
        it.R = p->rad[0];
        it.dmax = p->dmax[0];
        it.tab = p->tab;
        it.xt = p->xt;
        it.ns = (int)p->ns;
        int nh = 1;
        for (int q = 0; q < p->L - 1; ++q) nh *= p->rad[0];
        it.nh = nh;
        int sh = 1;
        for (int q = 0; q < p->m - 1; ++q) sh *= p->rad[0];
        it.stride_h = sh;
        it.stride_a = sh * nh;
        it.max_sweeps = r->opts.max_sweeps > 0 ? r->opts.max_sweeps : r->opts.fixed_sweeps;
        it.fixed = r->opts.fixed_sweeps;
        it.fp32 = r->opts.precision != PVI_FP64;
        it.gamma = p->d.gamma;
        it.cvar = p->d.c_var[0];
        it.thr = r->opts.eps * (1.0 - p->d.gamma) / p->d.gamma;
        auto* dd = reinterpret_cast<double*>(dptr(hb));
        it.pmf = dd;
        it.cdf = dd + p->tab;
        it.tail = dd + 2 * p->tab;
        it.r0 = dd + 3 * p->tab;
        it.v = reinterpret_cast<double*>(dptr(hb + o_v));
        it.gap = reinterpret_cast<double*>(dptr(hb + o_gap));
        it.stats = reinterpret_cast<double*>(dptr(hb + o_st));
        it.pi = reinterpret_cast<int32_t*>(dptr(hb + o_pi));
        items[k] = it;
    }

    int collect(int k, pvi::srv::Job* j) override {
        auto* r = static_cast<Request*>(j);
        pvi_mdp* p = r->mdp;
        const char* hb = arena(k);
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
        const int64_t sw = res.sweeps_fp32 + res.sweeps_fp64 + 1;
        res.logical_backups = p->logical_per_sweep * sw;
        res.executed_terms = p->executed_per_sweep * sw;
        res.vhat_shift = pvi::vhat_shift(p->d.gamma, res.dmax, res.dmin);
        res.status = stt[5] == 0.0 ? PVI_OK : PVI_E_NOT_CONVERGED;
        return res.status;
    }

    bool launch() override {
        if (pvi::launch_slots(dptr(hdr), dptr(sync), dptr(items), nslots, threads, lds, stream) !=
                hipSuccess ||
            hipEventRecord(done_ev, stream) != hipSuccess)
            return false;
        launched = true;
        return true;
    }
    bool finished() override { return !launched || hipEventQuery(done_ev) == hipSuccess; }
    void wait() override {
        if (launched) (void)hipEventSynchronize(done_ev);
    }
};

// Threads per slot work group, timed at the first server of a process: every slot is
// filled with a copy of a small instance of the serving family (m = 3, L = 1, order
// cap 10, Poisson(4) demand: 1,331 states, FP32 schedule), the stop word is set so
// that each work group serves its slot once and returns, and the launch is timed at
// 64, 128 and 256 threads; the fastest is kept for the process.  The size does not
// change any result.  PVI_SLOT_THREADS=64|128|256 fixes it; PVI_TUNE=0 keeps 256.
int slot_threads(HipSlotOps& ops) {
    if (const char* f = std::getenv("PVI_SLOT_THREADS")) {
        const int t = std::atoi(f);
        if (t == 64 || t == 128 || t == 256) return t;
    }
    const char* env = std::getenv("PVI_TUNE");
    if (env && std::strcmp(env, "0") == 0) return 256;
    static std::mutex mu;
    static int chosen = 0;
    std::lock_guard<std::mutex> lk(mu);
    if (chosen) return chosen;
    pvi_mdp_desc d{};
    d.struct_size = sizeof(d);
    d.family = PVI_FAMILY_LEADTIME;
    d.m = 3;
    d.lead_time = 1;
    d.n_periods = 1;
    d.a_max[0] = 10;
    d.d_max[0] = 20;
    d.demand_kind[0] = PVI_DEMAND_POISSON;
    d.demand_mean[0][0] = 4.0;
    d.c_var[0] = 3.0;
    d.c_hold = 1.0;
    d.c_short = 5.0;
    d.c_waste = 7.0;
    d.gamma = 0.99;
    d.issuing = PVI_FIFO;
    pvi_mdp* m = nullptr;
    if (mdp_create(&d, &m) != PVI_OK) return 256;
    Request r;
    r.mdp = m;
    r.opts.struct_size = sizeof(pvi_solve_opts);
    r.opts.precision = PVI_FP32;
    r.opts.eps = 1e-4;
    r.opts.max_sweeps = 100000;
    for (int k = 0; k < ops.nslots; ++k) ops.prepare(k, &r);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float best = 1e30f;
    int pick = 256;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        for (int t : {256, 128, 64}) {
            ops.threads = t;
            for (int k = 0; k < ops.nslots; ++k)
                __atomic_store_n(&ops.sync[k].seq, ops.sync[k].seq + 1, __ATOMIC_RELEASE);
            __atomic_store_n(&ops.hdr->stop, 1u, __ATOMIC_RELEASE);
            float ms = 0.f;
            if (hipEventRecord(e0, ops.stream) != hipSuccess || !ops.launch() ||
                hipEventRecord(e1, ops.stream) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                break;
            if (ms < best) {
                best = ms;
                pick = t;
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    __atomic_store_n(&ops.hdr->stop, 0u, __ATOMIC_RELEASE);
    mdp_destroy(m);
    const char* verbose = std::getenv("PVI_TUNE_VERBOSE");
    if (verbose && std::strcmp(verbose, "1") == 0)
        std::fprintf(stderr, "pvi: slot kernel %d threads per slot (%.2f ms for %d solves)\n",
                     pick, best, ops.nslots);
    chosen = pick;
    return pick;
}

void slot_feeder(pvi_server* S) {
    (void)hipSetDevice(S->device);
    pvi::srv::SlotConfig cfg;
    cfg.nslots = S->slots->nslots;
    cfg.worker = 0;
    cfg.launch_error_status = PVI_E_DEVICE;
    if (const char* e = std::getenv("PVI_SLOT_IDLE_MS")) cfg.idle_ms = std::max(1, std::atoi(e));
    pvi::srv::SlotFeeder feeder(*S->core, *S->slots, S->slots->hdr, S->slots->sync, cfg);
    feeder.run();
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
    int device = 0;
    (void)hipGetDevice(&device);
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess)
        return fail(PVI_E_DEVICE, "hipMemGetInfo failed");
    pvi::srv::Config cfg;
    cfg.budget = hbm_budget_bytes > 0 ? hbm_budget_bytes : (int64_t)(0.8 * (double)fr);
    cfg.log_path = std::getenv("PVI_SERVER_LOG");
    auto* S = new pvi_server();
    S->device = device;
    S->core = std::make_unique<pvi::srv::Core>(cfg);
    S->small_batch = small_batch > 0 ? small_batch : 256;
    if (small_batch > 0) {
        // as many slots as asked for, but no more than stay resident at once: every slot
        // needs a running work group
        int cap = pvi::slot_capacity(256, kSmallMaxLds);
        if (cap <= 0) cap = 256;
        S->slots = std::make_unique<HipSlotOps>();
        if (!S->slots->init(std::min(S->small_batch, cap))) {
            delete S;
            return fail(PVI_E_NOMEM, "pvi_server_create: slot table allocation failed");
        }
        S->slots->threads = slot_threads(*S->slots);
        S->workers.emplace_back(slot_feeder, S);
    }
    for (int i = 0; i < 2; ++i) S->workers.emplace_back(large_worker, S, 2 + i);
    *out = S;
    return PVI_OK;
}

pvi_status pvi_server_destroy(pvi_server* S) {
    if (!S) return PVI_OK;
    // requests that have not started are cancelled; running ones finish
    S->core->shutdown(PVI_E_CANCELLED);
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
    std::vector<std::unique_ptr<Job>> jobs;
    jobs.reserve(n);
    for (int i = 0; i < n; ++i) {
        auto r = std::make_unique<Request>();
        r->mdp = mdps[i];
        r->opts = *opts;
        r->opts.stream = nullptr;
        if (opts->v0) r->v0.assign(opts->v0, opts->v0 + mdps[i]->ns);
        r->small = S->small_batch > 0 && is_small(mdps[i], *opts);
        r->bytes = r->small ? 0 : (int64_t)pvi::device_bytes(mdps[i]);
        r->resident = mdps[i]->dev.ready;
        jobs.push_back(std::move(r));
    }
    if (!S->core->submit(jobs, tickets))
        return fail(PVI_E_CANCELLED, "vi_batch_submit: server is shutting down");
    return PVI_OK;
}

// A finished request's result; wall_ms is its latency (submit to done).
static void copy_result(const Request* q, pvi_result* res) {
    if (!res) return;
    *res = q->res;
    res->status = q->status;
    res->wall_ms = std::chrono::duration<double, std::milli>(q->t_done - q->t_submit).count();
}

pvi_status vi_poll(pvi_server* S, uint64_t ticket, pvi_result* res) {
    if (!S) return fail(PVI_E_INVALID, "vi_poll: NULL server");
    Job* j = nullptr;
    const int r = S->core->poll(ticket, &j);
    if (r < 0) return fail(PVI_E_INVALID, "vi_poll: unknown ticket");
    if (r == 0) return PVI_E_NOT_READY;
    auto* q = static_cast<Request*>(j);
    copy_result(q, res);
    return (pvi_status)q->status;
}

pvi_status vi_wait(pvi_server* S, uint64_t ticket, int64_t timeout_us, pvi_result* res) {
    if (!S) return fail(PVI_E_INVALID, "vi_wait: NULL server");
    Job* j = nullptr;
    const int r = S->core->wait(ticket, timeout_us, &j);
    if (r < 0) return fail(PVI_E_INVALID, "vi_wait: unknown ticket");
    if (r == 0) return PVI_E_NOT_READY;
    auto* q = static_cast<Request*>(j);
    copy_result(q, res);
    return (pvi_status)q->status;
}

pvi_status vi_ticket_info(pvi_server* S, uint64_t ticket, pvi_ticket_info* out) {
    if (!S || !out) return fail(PVI_E_INVALID, "vi_ticket_info: NULL argument");
    const bool known = S->core->visit(ticket, [&](const Job& j) {
        const auto& q = static_cast<const Request&>(j);
        std::memset(out, 0, sizeof(*out));
        out->state = j.state;
        out->small = j.small ? 1 : 0;
        out->worker = j.worker;
        out->sweeps = q.sweeps.load();
        out->status = j.state == pvi::srv::kDone ? j.status : PVI_E_NOT_READY;
        out->launch = j.launch.load();
        out->bytes = j.bytes;
        out->t_submit_ms = S->core->ms_since_start(j.t_submit);
        out->t_start_ms = j.state >= pvi::srv::kRunning ? S->core->ms_since_start(j.t_start) : -1.0;
        out->t_done_ms = j.state == pvi::srv::kDone ? S->core->ms_since_start(j.t_done) : -1.0;
    });
    if (!known) return fail(PVI_E_INVALID, "vi_ticket_info: unknown ticket");
    return PVI_OK;
}

pvi_status pvi_server_stats(pvi_server* S, double* p50, double* p99, int64_t* completed) {
    if (!S) return fail(PVI_E_INVALID, "pvi_server_stats: NULL server");
    S->core->stats(p50, p99, completed);
    return PVI_OK;
}

}  // extern "C"
