// Descriptor validation, host tables and the small accessors of the C ABI.
#include "mdp.h"

#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "tables.h"

namespace pvi {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

pvi_status fail(pvi_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

static bool is_finite(double x) { return std::isfinite(x); }

// Scenario A expected one-day reward without the order cost, as a table over
// (X_1, total stock): sum_d P(d) (-C_h [X - d - W]^+ - C_s [d - X]^+ - C_w W),
// W = [X_1 - d]^+ (Appendix A, reward equation).
static void build_a_tables(pvi_mdp* p) {
    const int R = p->rad[0], dm = p->dmax[0];
    const auto& P = p->pmf[0];
    p->tab = dm + 2;
    p->a_pmf.assign(p->tab, 0.0);
    p->a_cdf.assign(p->tab, 1.0);
    p->a_tail.assign(p->tab, 0.0);
    double c = 0.0;
    for (int d = 0; d <= dm; ++d) {
        p->a_pmf[d] = P[d];
        c += P[d];
        p->a_cdf[d] = d == dm ? 1.0 : c;
    }
    // P(D >= j) summed from the top so small tails keep their digits
    double t = 0.0;
    for (int d = dm; d >= 0; --d) {
        t += P[d];
        p->a_tail[d] = t;
    }
    p->xt = p->m * (R - 1) + 1;
    p->a_r0.assign((size_t)R * p->xt, 0.0);
    const double ch = p->d.c_hold, cs = p->d.c_short, cw = p->d.c_waste;
    for (int x1 = 0; x1 < R; ++x1)
        for (int X = 0; X < p->xt; ++X) {
            double e = 0.0;
            for (int d = 0; d <= dm; ++d) {
                const int W = std::max(x1 - d, 0);
                const double r = -ch * std::max(X - d - W, 0) - cs * std::max(d - X, 0) - cw * W;
                e += P[d] * r;
            }
            p->a_r0[(size_t)x1 * p->xt + X] = e;
        }
    // multiply-adds the kernel runs per sweep: for every state and action,
    // min(K, d_max - X_1) + 1 terms (1 when K = 0), K = X_2 + ... + X_m
    const int nz_dig = std::max(p->m - 2, 0);
    std::vector<int64_t> cnt(1, 1);  // number of (X_m..X_3) with digit sum b
    for (int i = 0; i < nz_dig; ++i) {
        std::vector<int64_t> nx(cnt.size() + R - 1, 0);
        for (size_t b = 0; b < cnt.size(); ++b)
            for (int v = 0; v < R; ++v) nx[b + v] += cnt[b];
        cnt.swap(nx);
    }
    int64_t nh = 1;
    for (int i = 0; i < p->L - 1; ++i) nh *= R;
    const int r2 = p->m >= 2 ? R : 1;
    int64_t ex = 0;
    for (size_t b = 0; b < cnt.size(); ++b) {
        int64_t per = 0;
        for (int x2 = 0; x2 < r2; ++x2)
            for (int x1 = 0; x1 < R; ++x1) {
                const int N = (int)b + x2;
                const int kmax = N == 0 ? 0 : std::max(0, std::min(N, dm - x1));
                per += kmax + 1;
            }
        ex += cnt[b] * per;
    }
    p->executed_per_sweep = nh * ex * R;
    p->logical_per_sweep = p->ns * p->na * (int64_t)(dm + 1);
}

}  // namespace pvi

using namespace pvi;

extern "C" {

const char* pvi_last_error(void) { return pvi::g_err.c_str(); }

pvi_status mdp_create(const pvi_mdp_desc* desc, pvi_mdp** out) {
    if (!desc || !out) return fail(PVI_E_INVALID, "mdp_create: NULL argument");
    if (desc->struct_size < sizeof(pvi_mdp_desc))
        return fail(PVI_E_INVALID, "mdp_create: struct_size too small");
    const pvi_mdp_desc& d = *desc;
    if (d.family < 0 || d.family > 2) return fail(PVI_E_INVALID, "mdp_create: bad family");
    if (d.m < 1 || d.m > PVI_MAX_LIFE) return fail(PVI_E_INVALID, "mdp_create: m out of range");
    if (!(d.gamma > 0.0 && d.gamma < 1.0))
        return fail(PVI_E_INVALID, "mdp_create: gamma must be in (0, 1)");
    const double costs[] = {d.c_var[0], d.c_var[1], d.c_fixed, d.c_hold, d.c_short,
                            d.c_waste, d.c_rev[0], d.c_rev[1], d.subst_rho};
    for (double c : costs)
        if (!is_finite(c)) return fail(PVI_E_INVALID, "mdp_create: non-finite cost");
    const int nprod = d.family == PVI_FAMILY_SUBST2 ? 2 : 1;
    for (int k = 0; k < nprod; ++k) {
        if (d.a_max[k] < 0 || d.a_max[k] > 31)
            return fail(PVI_E_INVALID, "mdp_create: a_max must be in 0..31");
        if (d.d_max[k] < 0 || d.d_max[k] > 1000)
            return fail(PVI_E_INVALID, "mdp_create: d_max must be in 0..1000");
    }
    int P = 1;
    if (d.family == PVI_FAMILY_LEADTIME) {
        if (d.lead_time < 1) return fail(PVI_E_INVALID, "mdp_create: scenario A needs L >= 1");
        if (d.m + d.lead_time - 1 > 12)
            return fail(PVI_E_INVALID, "mdp_create: too many state digits");
    } else {
        if (d.lead_time != 0)
            return fail(PVI_E_INVALID, "mdp_create: scenarios B and C need L = 0");
    }
    if (d.family == PVI_FAMILY_RUL_WEEKDAY) {
        if (d.m < 2) return fail(PVI_E_INVALID, "mdp_create: scenario C needs m >= 2");
        if (d.n_periods < 1 || d.n_periods > PVI_MAX_PERIODS)
            return fail(PVI_E_INVALID, "mdp_create: n_periods must be in 1..7");
        P = d.n_periods;
    } else if (d.n_periods != 1 && d.n_periods != 0) {
        return fail(PVI_E_INVALID, "mdp_create: n_periods must be 1 for scenarios A and B");
    }
    if (d.family == PVI_FAMILY_SUBST2 && !(d.subst_rho >= 0.0 && d.subst_rho <= 1.0))
        return fail(PVI_E_INVALID, "mdp_create: subst_rho must be in [0, 1]");

    pvi_mdp* p = new (std::nothrow) pvi_mdp();
    if (!p) return fail(PVI_E_NOMEM, "mdp_create: out of host memory");
    p->d = d;
    p->d.demand_table[0] = p->d.demand_table[1] = nullptr;
    p->family = d.family;
    p->m = d.m;
    p->L = d.lead_time;
    p->P = P;
    for (int k = 0; k < 2; ++k) {
        p->rad[k] = (k < nprod ? d.a_max[k] : 0) + 1;
        p->dmax[k] = k < nprod ? d.d_max[k] : 0;
    }
    // state digits, most significant first
    if (d.family == PVI_FAMILY_LEADTIME) {
        p->ndig = d.m + d.lead_time - 1;
        for (int i = 0; i < p->ndig; ++i) p->radix[i] = p->rad[0];
    } else if (d.family == PVI_FAMILY_SUBST2) {
        p->ndig = 2 * (d.m - 1);
        for (int i = 0; i < d.m - 1; ++i) {
            p->radix[i] = p->rad[0];
            p->radix[d.m - 1 + i] = p->rad[1];
        }
    } else {
        p->ndig = d.m;
        p->radix[0] = P;
        for (int i = 1; i < d.m; ++i) p->radix[i] = p->rad[0];
    }
    p->ns = 1;
    for (int i = 0; i < p->ndig; ++i) {
        p->ns *= p->radix[i];
        if (p->ns > (int64_t(1) << 31)) {
            delete p;
            return fail(PVI_E_INVALID, "mdp_create: more than 2^31 states");
        }
    }
    p->na = d.family == PVI_FAMILY_SUBST2 ? p->rad[0] * p->rad[1] : p->rad[0];
    // demand PMFs
    std::string err;
    for (int k = 0; k < nprod; ++k) {
        p->pmf[k].clear();
        for (int t = 0; t < P; ++t) {
            std::vector<double> row;
            const double* tb = d.demand_table[k] ? d.demand_table[k] + (size_t)t * (d.d_max[k] + 1)
                                                 : nullptr;
            const int tt = t < PVI_MAX_PERIODS ? t : 0;
            if (!demand_row(d.demand_kind[k], d.demand_mean[k][tt], d.demand_shape[k][tt],
                            d.d_max[k], tb, row, err)) {
                delete p;
                return fail(PVI_E_INVALID, "mdp_create: demand: " + err);
            }
            p->pmf[k].insert(p->pmf[k].end(), row.begin(), row.end());
        }
    }
    // remaining-life probabilities (Appendix C, age-on-arrival equations)
    if (d.family == PVI_FAMILY_RUL_WEEKDAY) {
        const int A = d.a_max[0];
        p->life.assign((size_t)(A + 1) * d.m, 0.0);
        for (int a = 0; a <= A; ++a) {
            double lg[PVI_MAX_LIFE], mx = 0.0;
            lg[0] = 0.0;
            for (int k = 2; k <= d.m; ++k) {
                lg[k - 1] = d.rul_c0[k - 1] + d.rul_c1[k - 1] * a;
                if (!is_finite(lg[k - 1])) {
                    delete p;
                    return fail(PVI_E_INVALID, "mdp_create: non-finite life logit");
                }
                mx = std::max(mx, lg[k - 1]);
            }
            double s = 0.0;
            for (int k = 0; k < d.m; ++k) s += std::exp(lg[k] - mx);
            for (int k = 0; k < d.m; ++k)
                p->life[(size_t)a * d.m + k] = std::exp(lg[k] - mx) / s;
        }
    }
    if (d.family == PVI_FAMILY_LEADTIME) build_a_tables(p);
    *out = p;
    return PVI_OK;
}

pvi_status mdp_destroy(pvi_mdp* mdp) {
    if (!mdp) return PVI_OK;
    pvi::free_device(mdp);
    delete mdp;
    return PVI_OK;
}

int64_t mdp_num_states(const pvi_mdp* mdp) { return mdp ? mdp->ns : -1; }
int32_t mdp_num_actions(const pvi_mdp* mdp) { return mdp ? mdp->na : -1; }
int32_t mdp_num_digits(const pvi_mdp* mdp) { return mdp ? mdp->ndig : -1; }

pvi_status mdp_encode(const pvi_mdp* p, const int32_t* digits, int64_t* idx) {
    if (!p || !digits || !idx) return fail(PVI_E_INVALID, "mdp_encode: NULL argument");
    int64_t v = 0;
    for (int i = 0; i < p->ndig; ++i) {
        if (digits[i] < 0 || digits[i] >= p->radix[i])
            return fail(PVI_E_INVALID, "mdp_encode: digit out of range");
        v = v * p->radix[i] + digits[i];
    }
    *idx = v;
    return PVI_OK;
}

pvi_status mdp_decode(const pvi_mdp* p, int64_t idx, int32_t* digits) {
    if (!p || !digits) return fail(PVI_E_INVALID, "mdp_decode: NULL argument");
    if (idx < 0 || idx >= p->ns) return fail(PVI_E_INVALID, "mdp_decode: index out of range");
    for (int i = p->ndig - 1; i >= 0; --i) {
        digits[i] = (int32_t)(idx % p->radix[i]);
        idx /= p->radix[i];
    }
    return PVI_OK;
}

pvi_status mdp_demand_pmf(const pvi_mdp* p, int32_t product, int32_t period, double* out) {
    if (!p || !out) return fail(PVI_E_INVALID, "mdp_demand_pmf: NULL argument");
    const int nprod = p->family == PVI_FAMILY_SUBST2 ? 2 : 1;
    if (product < 0 || product >= nprod || period < 0 || period >= p->P)
        return fail(PVI_E_INVALID, "mdp_demand_pmf: product or period out of range");
    const int n = p->dmax[product] + 1;
    std::memcpy(out, p->pmf[product].data() + (size_t)period * n, sizeof(double) * n);
    return PVI_OK;
}

pvi_status mdp_life_probs(const pvi_mdp* p, double* out) {
    if (!p || !out) return fail(PVI_E_INVALID, "mdp_life_probs: NULL argument");
    if (p->family != PVI_FAMILY_RUL_WEEKDAY)
        return fail(PVI_E_INVALID, "mdp_life_probs: only scenario C has life probabilities");
    std::memcpy(out, p->life.data(), sizeof(double) * p->life.size());
    return PVI_OK;
}

}  // extern "C"
