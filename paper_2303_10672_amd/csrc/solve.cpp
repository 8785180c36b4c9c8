// Device memory, the sweep loop with its precision schedule, and result access.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <string>
#include <vector>

#include "checkpoint.h"
#include "families.h"
#include "mdp.h"

namespace pvi {

size_t device_bytes(const pvi_mdp* p) {
    const size_t ns = (size_t)p->ns;
    size_t b = ns * (2 * sizeof(double) + 2 * sizeof(float) + sizeof(int32_t) + sizeof(double));
    b += family_extra_bytes(p);
    b += 4 * sizeof(double) * (size_t)family_tiles(p) + sizeof(Ctl) + 4096;
    // value tables the periodic stopping rule keeps beyond the two ping-pong ones
    if (p->P > 1) b += sizeof(double) * ((size_t)(p->P - 1) * ns + 2 * kPeriodicBlocks);
    return b;
}

void free_device(pvi_mdp* p) {
    auto& d = p->dev;
    if (!d.ready) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(d.device);
    if (d.own) (void)hipStreamSynchronize(d.own);
    void* bufs[] = {d.v64[0], d.v64[1], d.v32[0], d.v32[1], d.pi,  d.gap,
                    d.partials, d.ctl, d.pmf,   d.cdf,   d.tail, d.r0};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    for (double*& b : d.vring)
        if (b) {
            (void)hipFree(b);
            b = nullptr;
        }
    if (d.pparts) (void)hipFree(d.pparts);
    d.pparts = nullptr;
    family_free(p);
    if (d.h_ctl) (void)hipHostFree(d.h_ctl);
    for (auto e : d.ev) (void)hipEventDestroy(e);
    for (auto e : d.span_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& g : d.graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (d.own) (void)hipStreamDestroy(d.own);
    (void)hipSetDevice(prev);
    d = pvi_mdp::Dev{};
}

template <class T>
static hipError_t upload(T** dst, const std::vector<T>& src) {
    hipError_t e = hipMalloc((void**)dst, sizeof(T) * std::max<size_t>(src.size(), 1));
    if (e != hipSuccess) return e;
    if (src.empty()) return hipSuccess;
    return hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
}

static bool device_is_gfx950(int dev, std::string& name) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
    name = prop.gcnArchName;
    return name.rfind("gfx950", 0) == 0;
}

pvi_status ensure_device(pvi_mdp* p) {
    auto& d = p->dev;
    if (d.ready) {
        int cur = -1;
        PVI_HIP(hipGetDevice(&cur));
        if (cur != d.device) PVI_HIP(hipSetDevice(d.device));
        return PVI_OK;
    }
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0)
        return fail(PVI_E_DEVICE, "no HIP device available (this library has no CPU path)");
    int dev = 0;
    PVI_HIP(hipGetDevice(&dev));
    std::string arch;
    if (!device_is_gfx950(dev, arch))
        return fail(PVI_E_DEVICE, "device architecture " + arch + " is not gfx950");
    d.device = dev;
    const size_t ns = (size_t)p->ns;
    auto alloc = [&](void** ptr, size_t bytes) -> bool {
        return hipMalloc(ptr, std::max<size_t>(bytes, 16)) == hipSuccess;
    };
    bool ok = alloc((void**)&d.v64[0], ns * 8) && alloc((void**)&d.v64[1], ns * 8) &&
              alloc((void**)&d.v32[0], ns * 4) && alloc((void**)&d.v32[1], ns * 4) &&
              alloc((void**)&d.pi, ns * 4) && alloc((void**)&d.gap, ns * 8);
    d.tiles = family_tiles(p);
    ok = ok && alloc((void**)&d.partials, 4 * sizeof(double) * (size_t)d.tiles) &&
         alloc((void**)&d.ctl, sizeof(Ctl));
    if (ok && p->family == PVI_FAMILY_LEADTIME) {
        ok = upload(&d.pmf, p->a_pmf) == hipSuccess && upload(&d.cdf, p->a_cdf) == hipSuccess &&
             upload(&d.tail, p->a_tail) == hipSuccess && upload(&d.r0, p->a_r0) == hipSuccess;
    }
    d.ready = true;  // so free_device releases whatever was taken
    if (!ok) {
        free_device(p);
        return fail(PVI_E_NOMEM, "device allocation failed");
    }
    pvi_status st = family_init(p);
    if (st != PVI_OK) {
        free_device(p);
        return st;
    }
    if (hipHostMalloc((void**)&d.h_ctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) {
        free_device(p);
        return fail(PVI_E_NOMEM, "pinned host allocation failed");
    }
    if (hipStreamCreateWithFlags(&d.own, hipStreamNonBlocking) != hipSuccess) {
        free_device(p);
        return fail(PVI_E_DEVICE, "stream creation failed");
    }
    d.bytes = device_bytes(p);
    return PVI_OK;
}

namespace {

struct Phase {
    bool fp32 = false;
    int kahan = 0;
    int fixed = 0;       // > 0: exactly this many sweeps, no stopping rule
    int max_sweeps = 0;
    int k0 = 4;          // sweeps in the first batch
    int kmax = 64;       // cap on sweeps per batch
    bool time = false;
    int ring = 2;        // FP64 value tables cycled through (period + 1 for the periodic rule)
    int period = 0;      // > 0: run the periodic test after every sweep from this many on
    int hist0 = 0;       // earlier sweeps whose tables sit in the ring (a resumed solve)
    bool graphs = true;  // replay captured sweep graphs where the loop allows it
    double gamma = 0.0, thr = 0.0;
    // checkpoints of FP64 sweeps: file, interval, sweeps done before the phase, rule
    const char* ckpt = nullptr;
    int ckpt_every = 0, sweeps0 = 0, rule = 0;
    double ckpt_thr = 0.0;  // stopping threshold recorded in the files
    // progress report: sweeps of the solve completed so far (earlier phases' plus
    // this one's), stored at every host check
    std::atomic<int>* progress = nullptr;
    int progress_base = 0;
};

struct PhaseOut {
    int sweeps = 0;
    double backup_ms = 0.0;
    int timed = 0;
    bool stopped = false;
};

// FP64 value table of slot k: the two ping-pong tables, then the ring's extras.
double* v64_slot(pvi_mdp* p, int k) { return k < 2 ? p->dev.v64[k] : p->dev.vring[k]; }

// Ring slot of the table `back` sweeps before sweep `i` of a phase.
int ring_slot(int i, int back, int ring) { return ((i - back) % ring + ring) % ring; }

// Write the checkpoint after `done` sweeps of an FP64 phase: the last table, and
// under the periodic rule the earlier ones its test reads.
pvi_status write_checkpoint(pvi_mdp* p, const Phase& ph, int done, bool stopped,
                            hipStream_t s) {
    // tables in the ring: those a resume loaded (hist0 before its first) and the
    // sweeps since
    const int n = ph.period > 0 ? std::min(ph.hist0 + done, ph.period) + 1 : 1;
    const double* t[PVI_MAX_PERIODS + 1];
    for (int j = 0; j < n; ++j) t[j] = v64_slot(p, ring_slot(done, j, ph.ring));
    // the control block the host read at its last check holds this sweep's increments
    const Ctl& h = *p->dev.h_ctl;
    CheckpointStats cs;
    cs.threshold = ph.ckpt_thr;
    cs.dmax = h.dmax;
    cs.dmin = h.dmin;
    cs.span = h.span;
    return checkpoint_store(p, ph.ckpt, ph.rule, ph.sweeps0 + done, stopped ? 1 : 0, cs, t, n,
                            s);
}

pvi_status ensure_ring(pvi_mdp* p, int ring) {
    auto& d = p->dev;
    for (int k = 2; k < ring; ++k)
        if (!d.vring[k] && hipMalloc((void**)&d.vring[k], sizeof(double) * (size_t)p->ns) !=
                               hipSuccess)
            return fail(PVI_E_NOMEM, "vi_solve: periodic-rule value tables do not fit");
    if (!d.pparts &&
        hipMalloc((void**)&d.pparts, sizeof(double) * 2 * kPeriodicBlocks) != hipSuccess)
        return fail(PVI_E_NOMEM, "vi_solve: periodic-rule partials do not fit");
    return PVI_OK;
}

pvi_status init_ctl(pvi_mdp* p, hipStream_t s, double thr, double c0, int rule) {
    Ctl h{};
    h.rule = rule;
    h.mu = 0.0;
    h.c = c0;
    h.best_span = INFINITY;
    h.thr = thr;
    h.floor32 = 4.0 * std::ldexp(1.0, -23);
    *p->dev.h_ctl = h;
    PVI_HIP(hipMemcpyAsync(p->dev.ctl, p->dev.h_ctl, sizeof(Ctl), hipMemcpyHostToDevice, s));
    return PVI_OK;
}

// Sweeps per captured graph: an even number, so every replay starts on the same
// ping-pong table.
constexpr int kGraphSweeps = 8;

// Launch the backup and span kernels of sweep `launched` (ping-pong tables; no
// events, no periodic test).
pvi_status launch_sweep(pvi_mdp* p, const Phase& ph, int launched, hipStream_t s) {
    auto& d = p->dev;
    const void* vin = ph.fp32 ? (const void*)d.v32[launched & 1] : v64_slot(p, launched & 1);
    void* vout = ph.fp32 ? (void*)d.v32[(launched + 1) & 1] : v64_slot(p, (launched + 1) & 1);
    PVI_HIP(family_backup(p, ph.fp32, ph.kahan, 0, ph.fixed > 0, vin, vout, s));
    if (!family_fused_span(p))
        PVI_HIP(launch_span(d.ctl, d.partials, d.tiles, ph.fp32 ? 1 : 0, ph.fixed > 0,
                            p->d.gamma, s));
    return PVI_OK;
}

// The instantiated graph of kGraphSweeps sweeps from an even sweep index, captured
// on stream s at first use.  Each sweep's launches read the device stop flag, so a
// replay after the stopping rule fired does no work; the host still checks the flag
// between replays, as between batches of direct launches.
pvi_status sweep_graph(pvi_mdp* p, const Phase& ph, hipStream_t s, hipGraphExec_t* out) {
    auto& d = p->dev;
    const int key = (ph.fp32 ? 1 : 0) | (ph.kahan << 1) | ((ph.fixed > 0 ? 1 : 0) << 2);
    for (auto& g : d.graphs)
        if (g.key == key) {
            *out = g.exec;
            return PVI_OK;
        }
    hipGraph_t graph = nullptr;
    PVI_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    pvi_status st = PVI_OK;
    for (int i = 0; i < kGraphSweeps && st == PVI_OK; ++i) st = launch_sweep(p, ph, i, s);
    const hipError_t ec = hipStreamEndCapture(s, &graph);
    if (st != PVI_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    PVI_HIP(ec);
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    PVI_HIP(ei);
    d.graphs.push_back({key, exec});
    *out = exec;
    return PVI_OK;
}

pvi_status run_phase(pvi_mdp* p, const Phase& ph, hipStream_t s, PhaseOut& out) {
    auto& d = p->dev;
    int launched = 0, k = ph.k0;
    double prev_span = -1.0, prev_crit = -1.0;
    int prev_sweeps = 0, last_ckpt = 0;
    const int limit = ph.fixed > 0 ? ph.fixed : ph.max_sweeps;
    if (ph.time && (int)d.ev.size() < 2 * ph.kmax) {
        // timing only: no system-scope fence when they complete (the control block
        // reaches the host through its own copy and stream synchronisation)
        for (int i = (int)d.ev.size(); i < 2 * ph.kmax; ++i) {
            hipEvent_t e;
            PVI_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
            d.ev.push_back(e);
        }
    }
    // graphs serve the plain ping-pong loop; timed runs and the periodic rule (whose
    // value tables rotate through a longer ring) launch directly
    const bool graphs = ph.graphs && !ph.time && ph.period == 0 && ph.ring == 2;
    while (launched < limit) {
        int n = std::min(k, limit - launched);
        const int before = d.h_ctl->sweeps;
        if (graphs && (launched & 1) == 0 && n >= kGraphSweeps) {
            n -= n % kGraphSweeps;
            hipGraphExec_t exec = nullptr;
            const pvi_status st = sweep_graph(p, ph, s, &exec);
            if (st != PVI_OK) return st;
            for (int i = 0; i < n; i += kGraphSweeps) PVI_HIP(hipGraphLaunch(exec, s));
            launched += n;
        } else {
            for (int i = 0; i < n; ++i) {
                const void* vin = ph.fp32 ? (const void*)d.v32[launched & 1]
                                          : v64_slot(p, ring_slot(launched, 0, ph.ring));
                void* vout = ph.fp32 ? (void*)d.v32[(launched + 1) & 1]
                                     : v64_slot(p, ring_slot(launched + 1, 0, ph.ring));
                PVI_HIP(family_backup(p, ph.fp32, ph.kahan, 0, ph.fixed > 0, vin, vout, s,
                                      ph.time ? d.ev[2 * i] : nullptr,
                                      ph.time ? d.ev[2 * i + 1] : nullptr));
                if (!family_fused_span(p))
                    PVI_HIP(launch_span(d.ctl, d.partials, d.tiles, ph.fp32 ? 1 : 0,
                                        ph.fixed > 0, p->d.gamma, s));
                ++launched;
                if (ph.period > 0 && launched + ph.hist0 >= ph.period) {
                    // V_{i-j} for j = 0..P, i = launched (a sweep that was skipped after
                    // the stop flag leaves its table untouched, and so does this check)
                    PeriodicArgs a{};
                    for (int j = 0; j <= ph.period; ++j)
                        a.v[j] = v64_slot(p, ring_slot(launched, j, ph.ring));
                    a.P = ph.period;
                    a.gamma = ph.gamma;
                    a.thr = ph.thr;
                    a.n = p->ns;
                    PVI_HIP(launch_periodic_check(d.ctl, a, d.pparts, s));
                }
            }
        }
        PVI_HIP(hipMemcpyAsync(d.h_ctl, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        PVI_HIP(hipStreamSynchronize(s));
        const Ctl& h = *d.h_ctl;
        if (ph.progress) ph.progress->store(ph.progress_base + h.sweeps);
        if (ph.time) {
            const int real = std::min(n, h.sweeps - before);  // launches that did work
            for (int i = 0; i < real; ++i) {
                float ms = 0.f;
                PVI_HIP(hipEventElapsedTime(&ms, d.ev[2 * i], d.ev[2 * i + 1]));
                out.backup_ms += ms;
                ++out.timed;
            }
        }
        if (h.stop) {
            out.stopped = true;
            break;
        }
        if (ph.ckpt && ph.ckpt_every > 0 && !ph.fp32 && h.sweeps - last_ckpt >= ph.ckpt_every) {
            const pvi_status st = write_checkpoint(p, ph, h.sweeps, false, s);
            if (st != PVI_OK) return st;
            last_ckpt = h.sweeps;
        }
        // size the next batch from the observed contraction of what the stopping rule
        // tests: max |V' - V| for the sup-norm rule, else the span (which, under
        // discounting, falls below the threshold long before the sup-norm does); the
        // FP32 phase also ends at the span floor
        const double crit = h.rule == 1 ? std::max(std::fabs(h.dmax), std::fabs(h.dmin)) : h.span;
        const int gap = h.sweeps - prev_sweeps;
        if (ph.fixed > 0) {
            k = std::min(ph.kmax, 2 * k);
        } else if (prev_crit > 0.0 && crit > 0.0 && crit < prev_crit && gap > 0) {
            const double rate = std::pow(crit / prev_crit, 1.0 / gap);
            // a threshold <= 0 never stops the solve: full batches
            double need =
                rate < 1.0 && h.thr > 0.0 ? std::log(h.thr / crit) / std::log(rate) : ph.kmax;
            if (ph.fp32 && prev_span > 0.0 && h.span > 0.0 && h.span < prev_span) {
                const double rs = std::pow(h.span / prev_span, 1.0 / gap);
                if (rs < 1.0)
                    need = std::min(need, std::log(h.floor32 * h.vabs / h.span) / std::log(rs));
            }
            k = (int)std::min<double>(ph.kmax, std::max(1.0, std::ceil(need)));
        } else {
            k = std::min(ph.kmax, 2 * k);
        }
        prev_span = h.span;
        prev_crit = crit;
        prev_sweeps = h.sweeps;
    }
    out.sweeps = d.h_ctl->sweeps;
    return PVI_OK;
}

double midrange(const double* v, int64_t n) {
    if (!v || n == 0) return 0.0;
    double lo = v[0], hi = v[0];
    for (int64_t i = 1; i < n; ++i) {
        lo = std::min(lo, v[i]);
        hi = std::max(hi, v[i]);
    }
    return 0.5 * (lo + hi);
}

}  // namespace
// Move the results of the last solve (V, policy, Q gap) into the handle's host
// vectors and give its device buffers back.  The request server calls this for
// handles whose device state its own request created, so completed requests do
// not pin HBM that waiting requests need.
pvi_status park_results(pvi_mdp* p) {
    std::lock_guard<std::mutex> lock(p->mu);
    if (!p->dev.ready || p->have_result != 1) return PVI_OK;
    PVI_HIP(hipSetDevice(p->dev.device));
    p->h_v.resize(p->ns);
    p->h_pi.resize(p->ns);
    p->h_gap.resize(p->ns);
    PVI_HIP(hipMemcpy(p->h_v.data(), v64_slot(p, p->ret_buf), sizeof(double) * p->ns,
                      hipMemcpyDeviceToHost));
    PVI_HIP(hipMemcpy(p->h_pi.data(), p->dev.pi, sizeof(int32_t) * p->ns, hipMemcpyDeviceToHost));
    PVI_HIP(hipMemcpy(p->h_gap.data(), p->dev.gap, sizeof(double) * p->ns,
                      hipMemcpyDeviceToHost));
    p->have_result = 2;
    free_device(p);
    return PVI_OK;
}

}  // namespace pvi

using namespace pvi;

extern "C" {

pvi_status vi_solve(pvi_mdp* p, const pvi_solve_opts* opts_in, pvi_result* res) {
    return pvi::solve_impl(p, opts_in, res, true, nullptr);
}

}  // extern "C"

// The solve behind vi_solve; the request server passes graphs = false so that its
// concurrent workers launch every sweep directly.
pvi_status pvi::solve_impl(pvi_mdp* p, const pvi_solve_opts* opts_in, pvi_result* res,
                           bool graphs, std::atomic<int>* progress) {
    if (!p || !opts_in) return fail(PVI_E_INVALID, "vi_solve: NULL argument");
    // callers built against the layout that ended at `time_kernels` are accepted;
    // fields past their struct_size read as zero
    if (opts_in->struct_size < offsetof(pvi_solve_opts, stop_rule))
        return fail(PVI_E_INVALID, "vi_solve: struct_size too small");
    pvi_solve_opts oc{};
    std::memcpy(&oc, opts_in, std::min<size_t>(opts_in->struct_size, sizeof(pvi_solve_opts)));
    const pvi_solve_opts* o = &oc;
    if (o->stop_rule != PVI_STOP_SPAN && o->stop_rule != PVI_STOP_SUPNORM &&
        o->stop_rule != PVI_STOP_PERIODIC)
        return fail(PVI_E_INVALID, "vi_solve: bad stop_rule");
    if (o->precision < PVI_FP64 || o->precision > PVI_FP32_WIDE)
        return fail(PVI_E_INVALID, "vi_solve: bad precision");
    if (!(o->eps > 0.0)) return fail(PVI_E_INVALID, "vi_solve: eps must be > 0");
    if (o->max_sweeps <= 0 && o->fixed_sweeps <= 0)
        return fail(PVI_E_INVALID, "vi_solve: max_sweeps must be > 0");
    if (o->fixed_sweeps < 0) return fail(PVI_E_INVALID, "vi_solve: fixed_sweeps < 0");
    if (!family_supported(p)) return fail(PVI_E_INVALID, "vi_solve: " + family_support_msg(p));
    if (o->checkpoint_every < 0 || (o->resume != 0 && o->resume != 1))
        return fail(PVI_E_INVALID, "vi_solve: checkpoint_every >= 0 and resume 0 or 1 required");
    if ((o->checkpoint_every > 0 || o->resume) && !o->checkpoint_path)
        return fail(PVI_E_INVALID, "vi_solve: checkpoints need checkpoint_path");
    const bool resumed = o->resume != 0;
    Checkpoint ck;
    pvi_status st = PVI_OK;
    if (resumed) {
        if ((st = checkpoint_load(p, o->checkpoint_path, true, ck)) != PVI_OK) return st;
        if (o->fixed_sweeps > 0 && ck.sweeps > o->fixed_sweeps)
            return fail(PVI_E_INVALID, "vi_solve: the checkpoint is past fixed_sweeps");
    }
    const int k0 = resumed ? ck.sweeps : 0;  // FP64 sweeps done before this call
    std::lock_guard<std::mutex> lock(p->mu);
    const auto t0 = std::chrono::steady_clock::now();
    st = ensure_device(p);
    if (st != PVI_OK) return st;
    auto& d = p->dev;
    hipStream_t s = o->stream ? (hipStream_t)o->stream : d.own;
    for (auto& e : d.span_ev)
        if (!e) PVI_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    PVI_HIP(hipEventRecord(d.span_ev[0], s));
    const double g = p->d.gamma;
    // span rule: eps (1 - gamma)/gamma; undiscounted (gamma = 1), span < eps as in
    // Appendix B's test
    const double thr =
        o->stop_rule == PVI_STOP_SPAN && g < 1.0 ? o->eps * (1.0 - g) / g : o->eps;
    const bool periodic = o->stop_rule == PVI_STOP_PERIODIC && o->fixed_sweeps <= 0;
    const int period = p->P > 0 ? p->P : 1;
    if (periodic && (st = ensure_ring(p, period + 1)) != PVI_OK) return st;
    const int max_sweeps = o->max_sweeps > 0 ? o->max_sweeps : o->fixed_sweeps;
    const int kmax = o->check_every > 0 ? o->check_every : 64;
    p->have_result = 0;

    // initial values: a checkpoint's tables (newest in ring slot 0, earlier ones
    // behind it), v0, the family's default
    double c0 = 0.0;
    int hist0 = 0;
    if (resumed) {
        const int ring = periodic ? period + 1 : 2;
        const int nt = std::min<int>((int)ck.tables.size(), ring);
        for (int j = 0; j < nt; ++j)
            PVI_HIP(hipMemcpyAsync(v64_slot(p, ring_slot(0, j, ring)), ck.tables[j].data(),
                                   sizeof(double) * p->ns, hipMemcpyHostToDevice, s));
        hist0 = periodic ? nt - 1 : 0;
    } else if (o->v0) {
        PVI_HIP(hipMemcpyAsync(d.v64[0], o->v0, sizeof(double) * p->ns, hipMemcpyHostToDevice, s));
        c0 = midrange(o->v0, p->ns);
    } else if (p->family == PVI_FAMILY_SUBST2_L1) {
        PVI_HIP(family_initial_values(p, d.v64[0], s));
        const auto mm = std::minmax_element(p->b1_rev.begin(), p->b1_rev.end());
        c0 = 0.5 * (*mm.first + *mm.second);
    } else {
        PVI_HIP(launch_fill(d.v64[0], 0.0, p->ns, s));
    }
    PhaseOut o32, o64;
    const bool fp32 = o->precision != PVI_FP64 && !resumed;  // a resume goes on in FP64
    const int kahan = o->precision == PVI_FP32 ? 1 : 0;
    if (fp32) {
        PVI_HIP(launch_to_f32(d.v64[0], d.v32[0], c0, p->ns, s));
        if ((st = init_ctl(p, s, thr, c0, o->stop_rule)) != PVI_OK) return st;
        Phase ph;
        ph.fp32 = true;
        ph.kahan = kahan;
        ph.fixed = o->fixed_sweeps;
        // under the periodic rule the test itself runs on FP64 sweeps and needs only
        // about a cycle or two of them: the FP32 phase is a short warm start
        ph.max_sweeps = periodic ? std::min(max_sweeps, 2 * period) : max_sweeps;
        ph.kmax = kmax;
        ph.graphs = graphs;
        ph.time = o->time_kernels != 0;
        ph.progress = progress;
        if ((st = run_phase(p, ph, s, o32)) != PVI_OK) return st;
        PVI_HIP(launch_to_f64(d.v32[o32.sweeps & 1], d.v64[0], d.ctl, p->ns, s));
    }
    const bool fp64_phase = !fp32 || o->fixed_sweeps <= 0;
    if (fp64_phase) {
        if ((st = init_ctl(p, s, thr, 0.0, o->stop_rule)) != PVI_OK) return st;
        Phase ph;
        ph.fixed = fp32 ? 0 : (o->fixed_sweeps > 0 ? o->fixed_sweeps - k0 : 0);
        ph.max_sweeps = max_sweeps - k0;
        ph.kmax = kmax;
        ph.graphs = graphs;
        ph.k0 = fp32 ? 1 : 4;
        ph.time = o->time_kernels != 0;
        if (periodic) {
            ph.ring = period + 1;
            ph.period = period;
            ph.gamma = g;
            ph.thr = thr;
        }
        ph.hist0 = hist0;
        ph.progress = progress;
        ph.progress_base = o32.sweeps;
        ph.ckpt = o->checkpoint_every > 0 ? o->checkpoint_path : nullptr;
        ph.ckpt_every = o->checkpoint_every;
        ph.sweeps0 = k0;
        ph.rule = o->stop_rule;
        ph.ckpt_thr = thr;
        // a resumed solve whose checkpoint already met the same stopping rule at a
        // threshold no larger than this one, or reached its fixed sweep count or the
        // sweep cap, runs no more sweeps (a file of version 1 holds no threshold: its
        // solve goes on sweeping, and stops at once if the rule holds)
        const bool done_before = resumed && o->fixed_sweeps <= 0 && ck.stopped &&
                                 ck.rule == o->stop_rule && ck.threshold <= thr;
        const bool nothing_left = o->fixed_sweeps > 0 ? ph.fixed <= 0 : ph.max_sweeps <= 0;
        if (done_before || nothing_left)
            o64.stopped = done_before;
        else if ((st = run_phase(p, ph, s, o64)) != PVI_OK)
            return st;
        p->ret_buf = ring_slot(o64.sweeps, 0, ph.ring);
        // (a resume that ran no sweep leaves its file as it was)
        if (ph.ckpt && !(resumed && o64.sweeps == 0) &&
            (st = write_checkpoint(p, ph, o64.sweeps, o64.stopped, s)) != PVI_OK)
            return st;
    } else {
        p->ret_buf = 0;
    }
    // policy and Q gap from one more FP64 backup of the returned V
    PVI_HIP(family_backup(p, 0, 0, 1, 0, v64_slot(p, p->ret_buf), nullptr, s));
    PVI_HIP(hipEventRecord(d.span_ev[1], s));
    PVI_HIP(hipStreamSynchronize(s));
    p->have_result = 1;
    const bool converged = o->fixed_sweeps > 0 || o64.stopped;
    if (res) {
        std::memset(res, 0, sizeof(*res));
        const Ctl& h = *d.h_ctl;
        res->status = converged ? PVI_OK : PVI_E_NOT_CONVERGED;
        res->sweeps_fp32 = o32.sweeps;
        res->sweeps_fp64 = fp64_phase ? k0 + o64.sweeps : 0;
        res->backup_launches[0] = o64.timed;
        res->backup_launches[1] = o32.timed;
        // a resume that ran no sweep reports the increments the file recorded
        const bool from_file = resumed && o64.sweeps == 0 && fp64_phase;
        res->final_span = from_file ? ck.span : h.span;
        res->threshold = thr;
        res->dmax = from_file ? ck.dmax : h.dmax;
        res->dmin = from_file ? ck.dmin : h.dmin;
        res->backup_ms[0] = o64.backup_ms;
        res->backup_ms[1] = o32.backup_ms;
        const int64_t sweeps = o32.sweeps + o64.sweeps + 1;  // run by this call
        res->logical_backups = p->logical_per_sweep * sweeps;
        res->executed_terms = p->executed_per_sweep * sweeps;
        res->wall_ms = std::chrono::duration<double, std::milli>(
                           std::chrono::steady_clock::now() - t0).count();
        res->vhat_shift = vhat_shift(g, res->dmax, res->dmin);
        float ms = 0.f;
        PVI_HIP(hipEventElapsedTime(&ms, d.span_ev[0], d.span_ev[1]));
        res->device_ms = ms;
    }
    if (!converged) return fail(PVI_E_NOT_CONVERGED, "vi_solve: max_sweeps reached");
    return PVI_OK;
}

extern "C" {

pvi_status vi_backup(pvi_mdp* p, int32_t precision, const double* v_in, double* v_out,
                     int32_t* policy, double* q_gap) {
    if (!p || !v_in) return fail(PVI_E_INVALID, "vi_backup: NULL argument");
    if (precision < PVI_FP64 || precision > PVI_FP32_WIDE)
        return fail(PVI_E_INVALID, "vi_backup: bad precision");
    if (!family_supported(p)) return fail(PVI_E_INVALID, "vi_backup: " + family_support_msg(p));
    std::lock_guard<std::mutex> lock(p->mu);
    pvi_status st = ensure_device(p);
    if (st != PVI_OK) return st;
    auto& d = p->dev;
    hipStream_t s = d.own;
    p->have_result = 0;
    PVI_HIP(hipMemcpyAsync(d.v64[0], v_in, sizeof(double) * p->ns, hipMemcpyHostToDevice, s));
    if (precision == PVI_FP64) {
        if ((st = init_ctl(p, s, -1.0, 0.0, PVI_STOP_SPAN)) != PVI_OK) return st;
        PVI_HIP(family_backup(p, 0, 0, 0, 1, d.v64[0], d.v64[1], s));
        if (!family_fused_span(p))
            PVI_HIP(launch_span(d.ctl, d.partials, d.tiles, 0, 1, p->d.gamma, s));
    } else {
        const double c0 = midrange(v_in, p->ns);
        PVI_HIP(launch_to_f32(d.v64[0], d.v32[0], c0, p->ns, s));
        if ((st = init_ctl(p, s, -1.0, c0, PVI_STOP_SPAN)) != PVI_OK) return st;
        PVI_HIP(family_backup(p, 1, precision == PVI_FP32, 0, 1, d.v32[0], d.v32[1], s));
        if (!family_fused_span(p))
            PVI_HIP(launch_span(d.ctl, d.partials, d.tiles, 1, 1, p->d.gamma, s));
        PVI_HIP(launch_to_f64(d.v32[1], d.v64[1], d.ctl, p->ns, s));
    }
    PVI_HIP(family_backup(p, 0, 0, 1, 0, d.v64[0], nullptr, s));
    if (v_out)
        PVI_HIP(hipMemcpyAsync(v_out, d.v64[1], sizeof(double) * p->ns, hipMemcpyDeviceToHost, s));
    if (policy)
        PVI_HIP(hipMemcpyAsync(policy, d.pi, sizeof(int32_t) * p->ns, hipMemcpyDeviceToHost, s));
    if (q_gap)
        PVI_HIP(hipMemcpyAsync(q_gap, d.gap, sizeof(double) * p->ns, hipMemcpyDeviceToHost, s));
    PVI_HIP(hipStreamSynchronize(s));
    return PVI_OK;
}

pvi_status policy_get(const pvi_mdp* cp, int32_t* policy, double* q_gap) {
    pvi_mdp* p = const_cast<pvi_mdp*>(cp);
    if (!p || !policy) return fail(PVI_E_INVALID, "policy_get: NULL argument");
    std::lock_guard<std::mutex> lock(p->mu);
    if (!p->have_result) return fail(PVI_E_NOT_READY, "policy_get: no solve has completed");
    if (p->have_result == 2) {
        std::memcpy(policy, p->h_pi.data(), sizeof(int32_t) * p->ns);
        if (q_gap) std::memcpy(q_gap, p->h_gap.data(), sizeof(double) * p->ns);
        return PVI_OK;
    }
    PVI_HIP(hipSetDevice(p->dev.device));
    PVI_HIP(hipMemcpy(policy, p->dev.pi, sizeof(int32_t) * p->ns, hipMemcpyDeviceToHost));
    if (q_gap) PVI_HIP(hipMemcpy(q_gap, p->dev.gap, sizeof(double) * p->ns, hipMemcpyDeviceToHost));
    return PVI_OK;
}

pvi_status value_get(const pvi_mdp* cp, double* v) {
    pvi_mdp* p = const_cast<pvi_mdp*>(cp);
    if (!p || !v) return fail(PVI_E_INVALID, "value_get: NULL argument");
    std::lock_guard<std::mutex> lock(p->mu);
    if (!p->have_result) return fail(PVI_E_NOT_READY, "value_get: no solve has completed");
    if (p->have_result == 2) {
        std::memcpy(v, p->h_v.data(), sizeof(double) * p->ns);
        return PVI_OK;
    }
    PVI_HIP(hipSetDevice(p->dev.device));
    PVI_HIP(hipMemcpy(v, v64_slot(p, p->ret_buf), sizeof(double) * p->ns, hipMemcpyDeviceToHost));
    return PVI_OK;
}

pvi_status policy_get_device(const pvi_mdp* cp, int32_t* d_policy, void* stream) {
    pvi_mdp* p = const_cast<pvi_mdp*>(cp);
    if (!p || !d_policy) return fail(PVI_E_INVALID, "policy_get_device: NULL argument");
    std::lock_guard<std::mutex> lock(p->mu);
    if (!p->have_result) return fail(PVI_E_NOT_READY, "policy_get_device: no solve yet");
    if (p->have_result == 2) {
        hipStream_t s2 = (hipStream_t)stream;
        PVI_HIP(hipMemcpyAsync(d_policy, p->h_pi.data(), sizeof(int32_t) * p->ns,
                               hipMemcpyHostToDevice, s2));
        PVI_HIP(hipStreamSynchronize(s2));
        return PVI_OK;
    }
    PVI_HIP(hipSetDevice(p->dev.device));
    hipStream_t s = stream ? (hipStream_t)stream : p->dev.own;
    PVI_HIP(hipMemcpyAsync(d_policy, p->dev.pi, sizeof(int32_t) * p->ns,
                           hipMemcpyDeviceToDevice, s));
    if (!stream) PVI_HIP(hipStreamSynchronize(s));
    return PVI_OK;
}

}  // extern "C"
