// Host side of the rollout simulator: validation, the staged tables (demand CDFs
// summed left to right over the handle's PMFs, cumulative remaining-life
// probabilities), device buffers for one call, and the grid search of
// heuristic_search.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstddef>
#include <cstring>
#include <vector>

#include "mdp.h"
#include "pvi_internal.h"

using namespace pvi;

namespace {

// Buffers of one call, released on every path.
struct SimBuffers {
    std::vector<void*> ptrs;
    hipStream_t own = nullptr;
    ~SimBuffers() {
        if (own) {
            (void)hipStreamSynchronize(own);
            (void)hipStreamDestroy(own);
        }
        for (void* q : ptrs) (void)hipFree(q);
    }
    template <class T>
    hipError_t alloc(T** out, size_t n) {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, sizeof(T) * std::max<size_t>(n, 1));
        if (e == hipSuccess) ptrs.push_back(q);
        *out = static_cast<T*>(q);
        return e;
    }
};

pvi_status check_kind(const pvi_mdp* p, int kind) {
    if (kind == PVI_POLICY_TABLE) return PVI_OK;
    if (kind == PVI_POLICY_BASE_STOCK && p->family == PVI_FAMILY_LEADTIME) return PVI_OK;
    if (kind == PVI_POLICY_MOD_BASE_STOCK &&
        (p->family == PVI_FAMILY_SUBST2 || p->family == PVI_FAMILY_SUBST2_L1))
        return PVI_OK;
    if (kind == PVI_POLICY_S_S && p->family == PVI_FAMILY_RUL_WEEKDAY) return PVI_OK;
    return fail(PVI_E_INVALID, "policy_rollouts: the policy kind does not suit the family");
}

// Options up to and including `stream` are required; the per-product outputs
// that follow are read only when struct_size covers them.
constexpr size_t kOptsBase = offsetof(pvi_rollout_opts, product_kpis);

template <class T>
T opt_field(const pvi_rollout_opts* o, T pvi_rollout_opts::*f, size_t off) {
    return o->struct_size >= off + sizeof(T) ? o->*f : T{};
}

pvi_status run_rollouts(pvi_mdp* p, const pvi_rollout_opts* o, double* stats, double* returns,
                        double* kpis, const char* who) {
    const std::string w(who);
    if (!p || !o) return fail(PVI_E_INVALID, w + ": NULL argument");
    if (o->struct_size < kOptsBase)
        return fail(PVI_E_INVALID, w + ": struct_size too small");
    double* pkpis = opt_field(o, &pvi_rollout_opts::product_kpis,
                              offsetof(pvi_rollout_opts, product_kpis));
    double* pstats = opt_field(o, &pvi_rollout_opts::product_stats,
                               offsetof(pvi_rollout_opts, product_stats));
    if (o->kind < PVI_POLICY_TABLE || o->kind > PVI_POLICY_S_S)
        return fail(PVI_E_INVALID, w + ": bad policy kind");
    pvi_status st = check_kind(p, o->kind);
    if (st != PVI_OK) return st;
    const int n_pol = o->kind == PVI_POLICY_TABLE ? 1 : o->n_policies;
    if (o->kind == PVI_POLICY_TABLE && o->n_policies != 1)
        return fail(PVI_E_INVALID, w + ": a table policy needs n_policies = 1");
    if (n_pol < 1 || o->n_rollouts < 1 || o->warmup_days < 0 || o->horizon_days < 1)
        return fail(PVI_E_INVALID, w + ": n_policies, n_rollouts, horizon_days >= 1 and "
                                       "warmup_days >= 0 are required");
    if ((int64_t)n_pol * o->n_rollouts > 0x7fffffffLL)
        return fail(PVI_E_INVALID, w + ": n_policies x n_rollouts must stay below 2^31");
    if (o->warmup_days > (1 << 24) || o->horizon_days > (1 << 24))
        return fail(PVI_E_INVALID, w + ": more than 2^24 days");
    if (o->start_state < 0 || o->start_state >= p->ns)
        return fail(PVI_E_INVALID, w + ": start_state out of range");
    if (o->kind != PVI_POLICY_TABLE && !o->params)
        return fail(PVI_E_INVALID, w + ": a heuristic policy needs params");
    if (o->kind == PVI_POLICY_TABLE && p->ns > (int64_t(1) << 31))
        return fail(PVI_E_INVALID, w + ": a table policy needs at most 2^31 states");
    if (p->m > PVI_MAX_LIFE || (p->family == PVI_FAMILY_LEADTIME && p->L - 1 > 11))
        return fail(PVI_E_INVALID, w + ": state too long for the simulator");
    // Heuristic orders are not capped (scenario C's are), so a parameter bounds the
    // largest order; the per-rollout counts are 32-bit.
    int64_t qmax = std::max(p->d.a_max[0], p->d.a_max[1]);
    if (o->kind != PVI_POLICY_TABLE) {
        const int used = o->kind == PVI_POLICY_BASE_STOCK ? 1
                         : o->kind == PVI_POLICY_MOD_BASE_STOCK ? 2 : 14;
        for (int64_t i = 0; i < (int64_t)n_pol; ++i)
            for (int j = 0; j < used; ++j) {
                const int64_t v = o->params[i * PVI_POLICY_PARAMS + j];
                if (v > (1 << 20) || v < -(1 << 20))
                    return fail(PVI_E_INVALID, w + ": heuristic parameters must lie in "
                                                   "[-2^20, 2^20]");
                qmax = std::max(qmax, v);
            }
    }
    {
        const int64_t dsum = (int64_t)p->dmax[0] + (p->family == PVI_FAMILY_SUBST2 ||
                                                    p->family == PVI_FAMILY_SUBST2_L1
                                                ? p->dmax[1] : 0);
        const int64_t per_day = std::max<int64_t>(dsum, 2 * (int64_t)(p->m + p->L) * qmax);
        if ((int64_t)o->horizon_days * per_day > 0x7fffffffLL)
            return fail(PVI_E_INVALID, w + ": horizon_days too long for the 32-bit KPI counts "
                                           "at these order and demand sizes");
    }

    const bool two = p->family == PVI_FAMILY_SUBST2 || p->family == PVI_FAMILY_SUBST2_L1;
    if (!two && (pkpis || pstats))
        return fail(PVI_E_INVALID, w + ": per-product KPIs need a two-product family");
    const int R0 = p->rad[0], R1 = two ? p->rad[1] : 1;
    // demand CDFs, summed left to right over the PMF of each period
    const int P = p->family == PVI_FAMILY_RUL_WEEKDAY ? p->P : 1;
    std::vector<double> cdf0((size_t)P * (p->dmax[0] + 1)), cdf1;
    for (int t = 0; t < P; ++t) {
        double c = 0.0;
        for (int d = 0; d <= p->dmax[0]; ++d) {
            c += p->pmf[0][(size_t)t * (p->dmax[0] + 1) + d];
            cdf0[(size_t)t * (p->dmax[0] + 1) + d] = c;
        }
    }
    if (two) {
        cdf1.resize(p->dmax[1] + 1);
        double c = 0.0;
        for (int d = 0; d <= p->dmax[1]; ++d) cdf1[d] = c += p->pmf[1][d];
    }
    std::vector<double> lcum;
    if (p->family == PVI_FAMILY_RUL_WEEKDAY) {
        lcum.resize((size_t)R0 * p->m);
        for (int a = 0; a < R0; ++a) {
            double c = 0.0;
            for (int k = 0; k < p->m; ++k) lcum[(size_t)a * p->m + k] = c += p->life[(size_t)a * p->m + k];
        }
    }
    const size_t lds = sizeof(double) * (cdf0.size() + cdf1.size() + lcum.size());
    if (lds > 65536) return fail(PVI_E_INVALID, w + ": demand tables exceed LDS");

    // the policy table: the caller's, or the handle's last solved policy
    std::vector<int32_t> htab;
    const int32_t* dtab_src = nullptr;  // device policy of the handle
    if (o->kind == PVI_POLICY_TABLE) {
        if (o->table) {
            for (int64_t s = 0; s < p->ns; ++s)
                if (o->table[s] < 0 || o->table[s] >= p->na)
                    return fail(PVI_E_INVALID, w + ": table entry out of range");
            htab.assign(o->table, o->table + p->ns);
        } else {
            std::lock_guard<std::mutex> lock(p->mu);
            if (!p->have_result)
                return fail(PVI_E_NOT_READY, w + ": no solved policy on the handle");
            if (p->have_result == 2)
                htab = p->h_pi;
            else
                dtab_src = p->dev.pi;
        }
    }
    if (p->dev.ready) PVI_HIP(hipSetDevice(p->dev.device));

    SimBuffers B;
    hipStream_t s = static_cast<hipStream_t>(o->stream);
    if (!s) {
        PVI_HIP(hipStreamCreateWithFlags(&B.own, hipStreamNonBlocking));
        s = B.own;
    }
    SimDev d{};
    d.family = p->family == PVI_FAMILY_LEADTIME     ? 0
               : p->family == PVI_FAMILY_SUBST2       ? 1
               : p->family == PVI_FAMILY_RUL_WEEKDAY  ? 2
                                                      : 3;
    d.m = p->m;
    d.L = p->L;
    d.P = P;
    d.kind = o->kind;
    d.issuing = p->d.issuing;
    d.R0 = R0;
    d.R1 = R1;
    d.dmax0 = p->dmax[0];
    d.dmax1 = two ? p->dmax[1] : 0;
    d.n_pol = n_pol;
    d.n_roll = o->n_rollouts;
    d.warmup = o->warmup_days;
    d.horizon = o->horizon_days;
    d.n_cdf0 = (int)cdf0.size();
    d.n_cdf1 = (int)cdf1.size();
    d.n_lcum = (int)lcum.size();
    d.start = o->start_state;
    d.seed = o->seed;
    d.gamma = p->d.gamma;
    d.rho = p->d.subst_rho;
    d.mu0 = p->d.demand_mean[0][0];
    d.mu1 = p->d.demand_mean[1][0];
    d.cvar0 = p->d.c_var[0];
    d.cvar1 = p->d.c_var[1];
    d.cfixed = p->d.c_fixed;
    d.chold = p->d.c_hold;
    d.cshort = p->d.c_short;
    d.cwaste = p->d.c_waste;
    d.rev0 = p->d.c_rev[0];
    d.rev1 = p->d.c_rev[1];

    const size_t lanes = (size_t)n_pol * o->n_rollouts;
    const bool split = pkpis || pstats;
    double *dc0, *dc1, *dlc, *dret, *dkpi, *dstats, *dpkpi = nullptr, *dpstats = nullptr;
    int32_t *dprm = nullptr, *dtab = nullptr;
    if (B.alloc(&dc0, cdf0.size()) != hipSuccess || B.alloc(&dc1, cdf1.size()) != hipSuccess ||
        B.alloc(&dlc, lcum.size()) != hipSuccess || B.alloc(&dret, lanes) != hipSuccess ||
        B.alloc(&dkpi, 3 * lanes) != hipSuccess || B.alloc(&dstats, 8 * (size_t)n_pol) != hipSuccess)
        return fail(PVI_E_NOMEM, w + ": device allocation failed");
    if (split && (B.alloc(&dpkpi, 6 * lanes) != hipSuccess ||
                  B.alloc(&dpstats, 12 * (size_t)n_pol) != hipSuccess))
        return fail(PVI_E_NOMEM, w + ": device allocation failed");
    PVI_HIP(hipMemcpyAsync(dc0, cdf0.data(), sizeof(double) * cdf0.size(), hipMemcpyHostToDevice, s));
    if (!cdf1.empty())
        PVI_HIP(hipMemcpyAsync(dc1, cdf1.data(), sizeof(double) * cdf1.size(), hipMemcpyHostToDevice, s));
    if (!lcum.empty())
        PVI_HIP(hipMemcpyAsync(dlc, lcum.data(), sizeof(double) * lcum.size(), hipMemcpyHostToDevice, s));
    if (o->kind != PVI_POLICY_TABLE) {
        if (B.alloc(&dprm, (size_t)n_pol * PVI_POLICY_PARAMS) != hipSuccess)
            return fail(PVI_E_NOMEM, w + ": device allocation failed");
        PVI_HIP(hipMemcpyAsync(dprm, o->params, sizeof(int32_t) * n_pol * PVI_POLICY_PARAMS,
                               hipMemcpyHostToDevice, s));
    } else if (!dtab_src) {
        if (B.alloc(&dtab, (size_t)p->ns) != hipSuccess)
            return fail(PVI_E_NOMEM, w + ": device allocation failed");
        PVI_HIP(hipMemcpyAsync(dtab, htab.data(), sizeof(int32_t) * p->ns, hipMemcpyHostToDevice, s));
    }
    d.table = dtab_src ? dtab_src : dtab;
    d.params = dprm;
    d.cdf0 = dc0;
    d.cdf1 = dc1;
    d.lifecum = dlc;
    d.ret = dret;
    d.kpi = dkpi;
    d.pkpi = dpkpi;
    PVI_HIP(launch_rollouts(d, s));
    // stats[p] = (return, service, wastage, holding) x (mean, sd)
    PVI_HIP(launch_column_stats(dret, 1, 1, n_pol, o->n_rollouts, dstats, 8, 0, s));
    PVI_HIP(launch_column_stats(dkpi, 3, 3, n_pol, o->n_rollouts, dstats, 8, 2, s));
    if (split)
        PVI_HIP(launch_column_stats(dpkpi, 6, 6, n_pol, o->n_rollouts, dpstats, 12, 0, s));
    std::vector<double> hst(8 * (size_t)n_pol);
    PVI_HIP(hipMemcpyAsync(hst.data(), dstats, sizeof(double) * hst.size(), hipMemcpyDeviceToHost, s));
    if (returns)
        PVI_HIP(hipMemcpyAsync(returns, dret, sizeof(double) * lanes, hipMemcpyDeviceToHost, s));
    if (kpis)
        PVI_HIP(hipMemcpyAsync(kpis, dkpi, sizeof(double) * 3 * lanes, hipMemcpyDeviceToHost, s));
    if (pkpis)
        PVI_HIP(hipMemcpyAsync(pkpis, dpkpi, sizeof(double) * 6 * lanes, hipMemcpyDeviceToHost, s));
    if (pstats)
        PVI_HIP(hipMemcpyAsync(pstats, dpstats, sizeof(double) * 12 * n_pol, hipMemcpyDeviceToHost,
                               s));
    PVI_HIP(hipStreamSynchronize(s));
    if (stats) std::memcpy(stats, hst.data(), sizeof(double) * hst.size());
    return PVI_OK;
}

}  // namespace

extern "C" {

pvi_status policy_rollouts(pvi_mdp* p, const pvi_rollout_opts* o, double* stats, double* returns,
                           double* kpis) {
    return run_rollouts(p, o, stats, returns, kpis, "policy_rollouts");
}

pvi_status heuristic_search(pvi_mdp* p, const pvi_rollout_opts* o, double* stats, int32_t* best) {
    if (!p || !o || !best) return fail(PVI_E_INVALID, "heuristic_search: NULL argument");
    if (o->struct_size >= kOptsBase && o->kind == PVI_POLICY_TABLE)
        return fail(PVI_E_INVALID, "heuristic_search: needs a heuristic policy kind");
    const int n = o->n_policies;
    std::vector<double> st(8 * (size_t)std::max(n, 1));
    pvi_status rc = run_rollouts(p, o, st.data(), nullptr, nullptr, "heuristic_search");
    if (rc != PVI_OK) return rc;
    int b = 0;
    for (int i = 1; i < n; ++i)
        if (st[8 * (size_t)i] > st[8 * (size_t)b]) b = i;
    *best = b;
    if (stats) std::memcpy(stats, st.data(), sizeof(double) * 8 * n);
    return PVI_OK;
}

}  // extern "C"
