// vi_solve_noalloc: the FP64 scenario-A solve of vi_solve with no device
// allocation.  Its working memory (control block, tables, work list, span
// partials, the second value table) is the file-scope device array `scratch`; the
// caller brings the value, policy and gap outputs.  The kernels are the ones
// vi_solve launches, in the same order, so the results are bit-identical.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "families.h"
#include "mdp.h"

namespace {

// Layout of the scratch array (byte offsets; every region 256-byte aligned).
constexpr size_t kCtlBytes = 256;
constexpr size_t kTableBytes = size_t(512) << 10;     // pmf, cdf, tail, r0, work list
constexpr size_t kPartialBytes = size_t(512) << 10;   // span partials, 4 doubles each
constexpr int64_t kMaxStates = int64_t(1) << 22;      // 4,194,304 states
constexpr size_t kValueBytes = sizeof(double) * (size_t)kMaxStates;
constexpr size_t kScratchBytes = kCtlBytes + kTableBytes + kPartialBytes + kValueBytes;

}  // namespace

// The working memory of every vi_solve_noalloc call on a device (each device
// holds its own copy until the process ends).  Host code never passes this name
// to a kernel or a copy: it takes the device address from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu[kMaxDevices];           // one call at a time per device
char* g_scratch[kMaxDevices] = {};      // device address of `scratch`, per device
std::mutex g_init_mu;

// The device address of `scratch` on the current device, looked up at the first
// call on that device.
pvi_status scratch_ptr(int dev, char** out) {
    std::lock_guard<std::mutex> lk(g_init_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return pvi::fail(PVI_E_DEVICE, std::string("vi_solve_noalloc: hipGetSymbolAddress: ") +
                                               hipGetErrorString(e));
        g_scratch[dev] = static_cast<char*>(p);
    }
    *out = g_scratch[dev];
    return PVI_OK;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

using pvi::fail;

extern "C" pvi_status vi_solve_noalloc(const pvi_mdp* cp, const pvi_solve_opts* opts_in,
                                       double* d_v, int32_t* d_policy, double* d_gap,
                                       pvi_result* res) {
    pvi_mdp* p = const_cast<pvi_mdp*>(cp);
    if (!p || !opts_in || !d_v || !d_policy || !d_gap)
        return fail(PVI_E_INVALID, "vi_solve_noalloc: NULL argument");
    if (opts_in->struct_size < offsetof(pvi_solve_opts, stop_rule))
        return fail(PVI_E_INVALID, "vi_solve_noalloc: struct_size too small");
    pvi_solve_opts o{};
    std::memcpy(&o, opts_in, std::min<size_t>(opts_in->struct_size, sizeof(pvi_solve_opts)));
    if (p->family != PVI_FAMILY_LEADTIME)
        return fail(PVI_E_INVALID, "vi_solve_noalloc: scenario A (PVI_FAMILY_LEADTIME) only");
    if (o.precision != PVI_FP64)
        return fail(PVI_E_INVALID, "vi_solve_noalloc: PVI_FP64 only");
    if (o.stop_rule != PVI_STOP_SPAN && o.stop_rule != PVI_STOP_SUPNORM)
        return fail(PVI_E_INVALID, "vi_solve_noalloc: span or sup-norm stopping rule only");
    if (o.checkpoint_path || o.checkpoint_every != 0 || o.resume != 0)
        return fail(PVI_E_INVALID, "vi_solve_noalloc: no checkpoint files");
    if (!(o.eps > 0.0)) return fail(PVI_E_INVALID, "vi_solve_noalloc: eps must be > 0");
    if (o.fixed_sweeps < 0 || (o.max_sweeps <= 0 && o.fixed_sweeps <= 0))
        return fail(PVI_E_INVALID, "vi_solve_noalloc: max_sweeps > 0 or fixed_sweeps > 0");
    if (p->ns > kMaxStates)
        return fail(PVI_E_INVALID, "vi_solve_noalloc: " + std::to_string(p->ns) +
                                       " states exceed the limit of " +
                                       std::to_string(kMaxStates));
    const size_t tab = sizeof(double) * (size_t)p->tab;
    const size_t o_cdf = align256(tab), o_tail = o_cdf + align256(tab),
                 o_r0 = o_tail + align256(tab),
                 o_grp = o_r0 + align256(sizeof(double) * p->a_r0.size()),
                 t_end = o_grp + align256(sizeof(int32_t) * p->a_groups.size());
    const int tiles = pvi::family_tiles(p);
    if (t_end > kTableBytes || sizeof(double) * 4 * (size_t)tiles > kPartialBytes)
        return fail(PVI_E_INVALID, "vi_solve_noalloc: tables or work list exceed the "
                                   "scratch limits (512 KiB each)");

    int dev = 0;
    PVI_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PVI_E_DEVICE, "vi_solve_noalloc: device index");
    std::lock_guard<std::mutex> call_lock(g_mu[dev]);
    char* base = nullptr;
    pvi_status st = scratch_ptr(dev, &base);
    if (st != PVI_OK) return st;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)o.stream;
    auto* ctl = reinterpret_cast<pvi::Ctl*>(base);
    char* tb = base + kCtlBytes;
    auto* partials = reinterpret_cast<double*>(base + kCtlBytes + kTableBytes);
    auto* v_other = reinterpret_cast<double*>(base + kCtlBytes + kTableBytes + kPartialBytes);

    // tables and work list of this handle
    PVI_HIP(hipMemcpyAsync(tb, p->a_pmf.data(), tab, hipMemcpyHostToDevice, s));
    PVI_HIP(hipMemcpyAsync(tb + o_cdf, p->a_cdf.data(), tab, hipMemcpyHostToDevice, s));
    PVI_HIP(hipMemcpyAsync(tb + o_tail, p->a_tail.data(), tab, hipMemcpyHostToDevice, s));
    PVI_HIP(hipMemcpyAsync(tb + o_r0, p->a_r0.data(), sizeof(double) * p->a_r0.size(),
                           hipMemcpyHostToDevice, s));
    if (!p->a_groups.empty())
        PVI_HIP(hipMemcpyAsync(tb + o_grp, p->a_groups.data(),
                               sizeof(int32_t) * p->a_groups.size(), hipMemcpyHostToDevice, s));
    pvi::ADev a = pvi::make_adev(p);
    a.pmf = reinterpret_cast<const double*>(tb);
    a.cdf = reinterpret_cast<const double*>(tb + o_cdf);
    a.tail = reinterpret_cast<const double*>(tb + o_tail);
    a.r0 = reinterpret_cast<const double*>(tb + o_r0);
    a.groups = reinterpret_cast<const int32_t*>(tb + o_grp);
    a.ctl = ctl;
    a.partials = partials;
    a.pi = d_policy;
    a.gap = d_gap;

    // V_0 in the caller's table (slot 0); slot 1 is the scratch table
    double* slot[2] = {d_v, v_other};
    if (o.v0)
        PVI_HIP(hipMemcpyAsync(d_v, o.v0, sizeof(double) * p->ns, hipMemcpyHostToDevice, s));
    else
        PVI_HIP(pvi::launch_fill(d_v, 0.0, p->ns, s));
    const double g = p->d.gamma;
    const double thr = o.stop_rule == PVI_STOP_SPAN && g < 1.0 ? o.eps * (1.0 - g) / g : o.eps;
    // the control block starts like vi_solve's FP64 phase: every field rewritten,
    // since the array keeps the previous call's contents
    pvi::Ctl h{};
    h.rule = o.stop_rule;
    h.best_span = INFINITY;
    h.thr = thr;
    h.floor32 = 4.0 * std::ldexp(1.0, -23);
    PVI_HIP(hipMemcpyAsync(ctl, &h, sizeof(pvi::Ctl), hipMemcpyHostToDevice, s));
    PVI_HIP(hipStreamSynchronize(s));

    const bool fixed = o.fixed_sweeps > 0;
    const int limit = fixed ? o.fixed_sweeps : o.max_sweeps;
    const int kmax = o.check_every > 0 ? o.check_every : 64;
    auto backup = [&](const double* vin, double* vout, int extract) {
        a.v_in = vin;
        a.v_out = vout;
        a.fixed = fixed ? 1 : 0;
        return a.lifo ? pvi::launch_backup_a_lifo(a, 0, extract, s)
                      : pvi::launch_backup_a(a, 0, 0, extract, s);
    };
    // batches of direct launches between host checks of the stop flag; launches
    // after the flag is set return at once, so the batch sizes do not change V
    pvi::Ctl hc{};
    int launched = 0, k = 4;
    bool stopped = false;
    while (launched < limit) {
        const int n = std::min(k, limit - launched);
        for (int i = 0; i < n; ++i, ++launched) {
            PVI_HIP(backup(slot[launched & 1], slot[(launched + 1) & 1], 0));
            PVI_HIP(pvi::launch_span(ctl, partials, tiles, 0, fixed ? 1 : 0, g, s));
        }
        PVI_HIP(hipMemcpyAsync(&hc, ctl, sizeof(pvi::Ctl), hipMemcpyDeviceToHost, s));
        PVI_HIP(hipStreamSynchronize(s));
        if (hc.stop) {
            stopped = true;
            break;
        }
        k = std::min(kmax, 2 * k);
    }
    const int sweeps = hc.sweeps;
    // V after the last sweep that ran is in slot (sweeps & 1): the policy comes from
    // one more FP64 backup of it, and it ends in the caller's table
    PVI_HIP(backup(slot[sweeps & 1], nullptr, 1));
    if (sweeps & 1)
        PVI_HIP(hipMemcpyAsync(d_v, v_other, sizeof(double) * p->ns, hipMemcpyDeviceToDevice, s));
    PVI_HIP(hipStreamSynchronize(s));
    const bool converged = fixed || stopped;
    if (res) {
        std::memset(res, 0, sizeof(*res));
        res->status = converged ? PVI_OK : PVI_E_NOT_CONVERGED;
        res->sweeps_fp64 = sweeps;
        res->final_span = hc.span;
        res->threshold = thr;
        res->dmax = hc.dmax;
        res->dmin = hc.dmin;
        res->logical_backups = p->logical_per_sweep * (int64_t)(sweeps + 1);
        res->executed_terms = p->executed_per_sweep * (int64_t)(sweeps + 1);
        res->vhat_shift = pvi::vhat_shift(g, hc.dmax, hc.dmin);
        res->wall_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                .count();
    }
    if (!converged) return fail(PVI_E_NOT_CONVERGED, "vi_solve_noalloc: max_sweeps reached");
    return PVI_OK;
}
