// Host-side scenario tables, built once per MDP in FP64: demand PMFs with the
// folded tail, expected one-day rewards, remaining-life probabilities and the
// substitution-adjusted demand of product 1.
#include "tables.h"

#include <cmath>
#include <limits>

namespace pvi {

// Regularised incomplete gamma function.  Series expansion below a+1 and the
// Legendre continued fraction (evaluated with the modified Lentz method) above,
// as in Press et al., Numerical Recipes, section 6.2.
static double gamma_series(double a, double x) {
    double term = 1.0 / a, sum = term;
    for (int n = 1; n < 100000; ++n) {
        term *= x / (a + n);
        sum += term;
        if (std::fabs(term) <= std::fabs(sum) * 1e-17) break;
    }
    return sum * std::exp(-x + a * std::log(x) - std::lgamma(a));
}

static double gamma_cfrac(double a, double x) {
    const double tiny = 1e-300;
    double b = x + 1.0 - a, c = 1.0 / tiny, d = 1.0 / b, h = d;
    for (int i = 1; i < 100000; ++i) {
        const double an = -i * (i - a);
        b += 2.0;
        d = an * d + b;
        if (std::fabs(d) < tiny) d = tiny;
        c = b + an / c;
        if (std::fabs(c) < tiny) c = tiny;
        d = 1.0 / d;
        const double del = d * c;
        h *= del;
        if (std::fabs(del - 1.0) < 1e-16) break;
    }
    return std::exp(-x + a * std::log(x) - std::lgamma(a)) * h;
}

double gamma_p(double a, double x) {  // P(a, x) = lower / Gamma(a)
    if (x <= 0.0) return 0.0;
    if (x < a + 1.0) return gamma_series(a, x);
    return 1.0 - gamma_cfrac(a, x);
}

double gamma_q(double a, double x) {  // Q(a, x) = 1 - P(a, x)
    if (x <= 0.0) return 1.0;
    if (x < a + 1.0) return 1.0 - gamma_series(a, x);
    return gamma_cfrac(a, x);
}

static double poisson_pmf(int d, double mu) {
    if (mu <= 0.0) return d == 0 ? 1.0 : 0.0;
    return std::exp(d * std::log(mu) - mu - std::lgamma(d + 1.0));
}

static double negbin_pmf(int d, double n, double p) {
    return std::exp(std::lgamma(d + n) - std::lgamma(n) - std::lgamma(d + 1.0) +
                    n * std::log(p) + d * std::log1p(-p));
}

// Sum of a PMF from d0 upwards until the terms stop mattering (the folded tail).
template <class F>
static double upper_tail(F pmf, int d0) {
    double s = 0.0;
    for (int d = d0; d < d0 + 100000; ++d) {
        const double t = pmf(d);
        s += t;
        if (d > d0 + 8 && t <= s * 1e-18) break;
    }
    return s;
}

bool demand_row(int kind, double mean, double shape, int dmax, const double* table,
                std::vector<double>& out, std::string& err) {
    out.assign(dmax + 1, 0.0);
    switch (kind) {
        case PVI_DEMAND_NONE:
            out[0] = 1.0;
            return true;
        case PVI_DEMAND_POISSON: {
            if (!(mean >= 0.0)) return err = "poisson mean must be >= 0", false;
            for (int d = 0; d < dmax; ++d) out[d] = poisson_pmf(d, mean);
            out[dmax] = upper_tail([&](int d) { return poisson_pmf(d, mean); }, dmax);
            return true;
        }
        case PVI_DEMAND_GAMMA: {
            if (!(mean > 0.0) || !(shape > 0.0)) return err = "gamma needs mean, cv > 0", false;
            const double k = 1.0 / (shape * shape), theta = mean * shape * shape;
            auto F = [&](double x) { return x <= 0.0 ? 0.0 : gamma_p(k, x / theta); };
            for (int d = 0; d < dmax; ++d) out[d] = F(d + 0.5) - F(d - 0.5);
            out[dmax] = dmax == 0 ? 1.0 : gamma_q(k, (dmax - 0.5) / theta);
            return true;
        }
        case PVI_DEMAND_NEGBIN: {
            if (!(mean > 0.0) || !(shape > 0.0)) return err = "negbin needs mean, n > 0", false;
            const double p = shape / (shape + mean);
            for (int d = 0; d < dmax; ++d) out[d] = negbin_pmf(d, shape, p);
            out[dmax] = upper_tail([&](int d) { return negbin_pmf(d, shape, p); }, dmax);
            return true;
        }
        case PVI_DEMAND_TABLE: {
            if (!table) return err = "demand_table is NULL", false;
            double s = 0.0;
            for (int d = 0; d <= dmax; ++d) {
                if (!(table[d] >= 0.0)) return err = "demand_table has a negative entry", false;
                out[d] = table[d];
                s += table[d];
            }
            if (std::fabs(s - 1.0) > 1e-12) return err = "demand_table row does not sum to 1", false;
            return true;
        }
        default:
            return err = "unknown demand kind", false;
    }
}

double binom_pmf(int k, int n, double rho) {
    if (k < 0 || k > n) return 0.0;
    if (rho <= 0.0) return k == 0 ? 1.0 : 0.0;
    if (rho >= 1.0) return k == n ? 1.0 : 0.0;
    return std::exp(std::lgamma(n + 1.0) - std::lgamma(k + 1.0) - std::lgamma(n - k + 1.0) +
                    k * std::log(rho) + (n - k) * std::log1p(-rho));
}

}  // namespace pvi
