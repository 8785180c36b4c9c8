/*
 * Plain FP64 CPU value iteration for perishable-inventory MDPs: the ORACLE.
 *
 * Test infrastructure only.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this file's library.  It shares no source with the
 * GPU library and implements every step by its plain definition:
 *
 *   Q(s,a)   = sum over outcomes w of P(w|s,a) * (r_w + gamma * V(s'_w)),
 *              where (s'_w, r_w) = T(s, a, w)         (deterministic-transition
 *              form of the value-iteration update, Methods, "Value iteration")
 *   V'(s)    = max_a Q(s,a),  pi(s) = lowest argmax_a Q(s,a)
 *   stop     when max_s(V'-V) - min_s(V'-V) < eps*(1-gamma)/gamma
 *
 * Outcomes are enumerated one by one and summed left to right in outcome order;
 * nothing is factorised, hoisted or reordered.
 *
 * Scenario A (Appendix A, FIFO equation and reward equation): state
 *   [O_{L-1}, ..., O_1, X_m, ..., X_1], outcome = demand d.
 * Scenario B (Appendix B, FIFO equation and reward equation, substitution as in
 *   the Scenario B problem description): L = 0 here, state
 *   [A_{m-1}..A_1, B_{m-1}..B_1], outcome = (dA, dB, k) where k ~ Binomial(uA, rho)
 *   of product 0's unmet demand uA accept product 1, served from product 1's stock
 *   left after its own demand, oldest first.
 * Scenario B as the paper runs it (family 3; Appendix B): lead time 1, state
 *   [Xa_m..Xa_1, Xb_m..Xb_1], outcome = units issued (h_a, h_b), probabilities
 *   P(h_a, h_b | I_a, I_b) supplied as a table built from the demand and
 *   substitution definitions (oracle.py).
 * Scenario C (Appendix C, state-transition and reward equations): state
 *   [tau, X_{m-1}, ..., X_1], outcome = (d, y) with y a multinomial split of the
 *   order over remaining lives m..1 and stock of each life capped at a_max.
 *
 * Demand PMFs (with their folded tails) and remaining-life probabilities are
 * inputs; oracle.py builds them from the scenario parameters.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXD 16 /* max digits in a state */

typedef struct {
    int32_t family;      /* 0 = A, 1 = B, 2 = C */
    int32_t m, L, n_periods;
    int32_t a_max[2], d_max[2];
    const double* pmf0;  /* product 0 demand PMF, [n_periods][d_max[0]+1] */
    const double* pmf1;  /* product 1 demand PMF (B), [d_max[1]+1] */
    const double* rul_p; /* C: [a_max+1][m]; entry (a, k-1) = p_k(a), k = remaining life */
    double rho;
    double c_var[2], c_fixed, c_hold, c_short, c_waste, c_rev[2];
    double gamma;
    int32_t issuing;     /* A: 0 = FIFO (eq:demoor:fifo), 1 = LIFO (eq:demoor:lifo) */
    /* family 3 (Scenario B as the paper runs it): P(h_a, h_b | I_a, I_b), flattened
     * [I_a][I_b][h_a][h_b] with I_a, h_a in 0..m a_max[0], I_b, h_b in 0..m a_max[1] */
    const double* issue_p;
} or_mdp;

static double pos(double x) { return x > 0.0 ? x : 0.0; }
static int ipos(int x) { return x > 0 ? x : 0; }

/* ---------------------------------------------------------------- encoding */

static int n_digits(const or_mdp* p) {
    if (p->family == 0) return p->m + p->L - 1;
    if (p->family == 1) return 2 * (p->m - 1);
    if (p->family == 3) return 2 * p->m;
    return p->m; /* tau + (m-1) stock digits */
}

static void radices(const or_mdp* p, int* rad) {
    int n = n_digits(p);
    if (p->family == 0) {
        for (int i = 0; i < n; ++i) rad[i] = p->a_max[0] + 1;
    } else if (p->family == 1) {
        for (int i = 0; i < p->m - 1; ++i) rad[i] = p->a_max[0] + 1;
        for (int i = 0; i < p->m - 1; ++i) rad[p->m - 1 + i] = p->a_max[1] + 1;
    } else if (p->family == 3) {
        for (int i = 0; i < p->m; ++i) rad[i] = p->a_max[0] + 1;
        for (int i = 0; i < p->m; ++i) rad[p->m + i] = p->a_max[1] + 1;
    } else {
        rad[0] = p->n_periods;
        for (int i = 1; i < n; ++i) rad[i] = p->a_max[0] + 1;
    }
}

int64_t or_num_states(const or_mdp* p) {
    int rad[OR_MAXD];
    radices(p, rad);
    int64_t n = 1;
    for (int i = 0; i < n_digits(p); ++i) n *= rad[i];
    return n;
}

int32_t or_num_actions(const or_mdp* p) {
    if (p->family == 1 || p->family == 3) return (p->a_max[0] + 1) * (p->a_max[1] + 1);
    return p->a_max[0] + 1;
}

/* digits in written order, most significant first */
void or_decode(const or_mdp* p, int64_t idx, int32_t* dig) {
    int rad[OR_MAXD];
    radices(p, rad);
    for (int i = n_digits(p) - 1; i >= 0; --i) {
        dig[i] = (int32_t)(idx % rad[i]);
        idx /= rad[i];
    }
}

int64_t or_encode(const or_mdp* p, const int32_t* dig) {
    int rad[OR_MAXD];
    radices(p, rad);
    int64_t idx = 0;
    for (int i = 0; i < n_digits(p); ++i) idx = idx * rad[i] + dig[i];
    return idx;
}

/* -------------------------------------------------------------- scenario A */
/* One transition of Scenario A.  dig = [O_{L-1}..O_1, X_m..X_1]. */
static void trans_a(const or_mdp* p, const int32_t* dig, int a, int d, int32_t* nd,
                    double* r) {
    int m = p->m, L = p->L;
    int X[OR_MAXD + 1]; /* X[1..m] */
    int O[OR_MAXD + 1]; /* O[1..L-1] */
    for (int i = 1; i <= L - 1; ++i) O[i] = dig[(L - 1) - i];
    for (int j = 1; j <= m; ++j) X[j] = dig[(L - 1) + (m - j)];
    int Xtot = 0;
    for (int j = 1; j <= m; ++j) Xtot += X[j];
    int W, Xn[OR_MAXD + 1], On[OR_MAXD + 1];
    if (p->issuing == 1) {
        /* LIFO (eq:demoor:lifo): the youngest units go first; X_{j+1} meets the
           demand left after X_m .. X_{j+2}, and X_1 only what the others could not */
        int above = 0; /* X_2 + ... + X_m */
        for (int k = 2; k <= m; ++k) above += X[k];
        W = ipos(X[1] - ipos(d - above));
        for (int j = 1; j <= m - 1; ++j) {
            int younger = 0; /* X_{j+2} + ... + X_m */
            for (int k = j + 2; k <= m; ++k) younger += X[k];
            Xn[j] = ipos(X[j + 1] - ipos(d - younger));
        }
    } else {
        /* FIFO (eq:demoor:fifo): the oldest units go first */
        W = ipos(X[1] - d); /* units expiring at the end of the day */
        int cum = 0;
        for (int j = 1; j <= m - 1; ++j) {
            cum += X[j];
            Xn[j] = ipos(X[j + 1] - ipos(d - cum));
        }
    }
    Xn[m] = (L >= 2) ? O[1] : a;
    if (L >= 2) {
        On[L - 1] = a;
        for (int i = 1; i <= L - 2; ++i) On[i] = O[i + 1];
    }
    for (int i = 1; i <= L - 1; ++i) nd[(L - 1) - i] = On[i];
    for (int j = 1; j <= m; ++j) nd[(L - 1) + (m - j)] = Xn[j];
    *r = -p->c_var[0] * a - p->c_hold * pos((double)(Xtot - d - W)) -
         p->c_short * pos((double)(d - Xtot)) - p->c_waste * W;
}

static double q_a(const or_mdp* p, const double* V, const int32_t* dig, int a) {
    int32_t nd[OR_MAXD];
    double q = 0.0;
    for (int d = 0; d <= p->d_max[0]; ++d) {
        double pr = p->pmf0[d];
        if (pr == 0.0) continue;
        double r;
        trans_a(p, dig, a, d, nd, &r);
        q += pr * (r + p->gamma * V[or_encode(p, nd)]);
    }
    return q;
}

/* -------------------------------------------------------------- scenario B */
/* FIFO issue of demand e from stock o[1..m] (oldest first); returns units issued,
 * writes leftovers into left[1..m]. */
static int fifo_issue(const int* o, int m, int e, int* left) {
    int issued = 0;
    for (int j = 1; j <= m; ++j) {
        int take = e < o[j] ? e : o[j];
        left[j] = o[j] - take;
        e -= take;
        issued += take;
    }
    return issued;
}

static double binom_pmf(int k, int n, double rho) {
    if (k < 0 || k > n) return 0.0;
    /* n choose k by the product formula, then rho^k (1-rho)^(n-k) */
    double c = 1.0;
    for (int i = 1; i <= k; ++i) c = c * (double)(n - k + i) / (double)i;
    return c * pow(rho, (double)k) * pow(1.0 - rho, (double)(n - k));
}

/* dig = [A_{m-1}..A_1, B_{m-1}..B_1]; action (aA, aB); outcome (dA, dB, k). */
static void trans_b(const or_mdp* p, const int32_t* dig, int aA, int aB, int dA, int dB,
                    int k, int32_t* nd, double* r) {
    int m = p->m;
    int oA[OR_MAXD + 1], oB[OR_MAXD + 1], lA[OR_MAXD + 1], lB[OR_MAXD + 1];
    for (int j = 1; j <= m - 1; ++j) {
        oA[j] = dig[(m - 1) - j];
        oB[j] = dig[(m - 1) + (m - 1) - j];
    }
    oA[m] = aA; /* L = 0: today's order is on hand, with m days of life */
    oB[m] = aB;
    int hA = fifo_issue(oA, m, dA, lA);
    int uA = dA - hA;
    (void)uA;
    int lB1[OR_MAXD + 1];
    int hB_own = fifo_issue(oB, m, dB, lB1);
    int hB_sub = fifo_issue(lB1, m, k, lB); /* substitutes take what is left, FIFO */
    /* next state: units of life j+1 that were not issued now have life j;
     * life-1 leftovers expire */
    for (int j = 1; j <= m - 1; ++j) {
        nd[(m - 1) - j] = lA[j + 1];
        nd[(m - 1) + (m - 1) - j] = lB[j + 1];
    }
    *r = -(p->c_var[0] * aA + p->c_var[1] * aB) + p->c_rev[0] * hA +
         p->c_rev[1] * (hB_own + hB_sub);
}

static double q_b(const or_mdp* p, const double* V, const int32_t* dig, int aA, int aB) {
    int m = p->m;
    int32_t nd[OR_MAXD];
    int stockA = aA;
    for (int j = 0; j < m - 1; ++j) stockA += dig[j];
    double q = 0.0;
    for (int dA = 0; dA <= p->d_max[0]; ++dA) {
        double pA = p->pmf0[dA];
        if (pA == 0.0) continue;
        int uA = ipos(dA - stockA);
        for (int dB = 0; dB <= p->d_max[1]; ++dB) {
            double pB = p->pmf1[dB];
            if (pB == 0.0) continue;
            for (int k = 0; k <= uA; ++k) {
                double pk = binom_pmf(k, uA, p->rho);
                if (pk == 0.0) continue;
                double r;
                trans_b(p, dig, aA, aB, dA, dB, k, nd, &r);
                q += pA * pB * pk * (r + p->gamma * V[or_encode(p, nd)]);
            }
        }
    }
    return q;
}

/* ------------------------------------------- scenario B as the paper runs it */
/* Family 3 (Scenario B description and Appendix B): lead time 1, so the state
 * [Xa_m..Xa_1, Xb_m..Xb_1] includes yesterday's orders as X_m; the outcome is the
 * units issued (h_a, h_b); issuing is FIFO per product (FIFO equation of Appendix
 * B), today's order becomes tomorrow's X_m; reward -(C_v^a A^a + C_v^b A^b) +
 * C_r^a h_a + C_r^b h_b (reward equation, with the garbled C^a_v A^b read as
 * C^b_v A^b). */
static void trans_b1(const or_mdp* p, const int32_t* dig, int aA, int aB, int hA, int hB,
                     int32_t* nd, double* r) {
    int m = p->m;
    int xa[OR_MAXD + 1], xb[OR_MAXD + 1];
    for (int j = 1; j <= m; ++j) {
        xa[j] = dig[m - j];
        xb[j] = dig[m + (m - j)];
    }
    int ca = 0, cb = 0;
    for (int j = 1; j <= m - 1; ++j) {
        ca += xa[j];
        cb += xb[j];
        nd[m - j] = ipos(xa[j + 1] - ipos(hA - ca));
        nd[m + (m - j)] = ipos(xb[j + 1] - ipos(hB - cb));
    }
    nd[0] = aA;
    nd[m] = aB;
    *r = -(p->c_var[0] * aA + p->c_var[1] * aB) + p->c_rev[0] * hA + p->c_rev[1] * hB;
}

static double q_b1(const or_mdp* p, const double* V, const int32_t* dig, int aA, int aB) {
    int m = p->m;
    int Ia = 0, Ib = 0;
    for (int j = 0; j < m; ++j) {
        Ia += dig[j];
        Ib += dig[m + j];
    }
    int HA = m * p->a_max[0] + 1, HB = m * p->a_max[1] + 1;
    const double* P = p->issue_p + ((size_t)Ia * HB + Ib) * (size_t)HA * HB;
    int32_t nd[OR_MAXD];
    double q = 0.0;
    for (int hA = 0; hA <= Ia; ++hA)
        for (int hB = 0; hB <= Ib; ++hB) {
            double pr = P[(size_t)hA * HB + hB];
            if (pr == 0.0) continue;
            double r;
            trans_b1(p, dig, aA, aB, hA, hB, nd, &r);
            q += pr * (r + p->gamma * V[or_encode(p, nd)]);
        }
    return q;
}

/* -------------------------------------------------------------- scenario C */
/* dig = [tau, X_{m-1}..X_1]; y[1..m] arrivals by remaining life; demand d. */
static void trans_c(const or_mdp* p, const int32_t* dig, int a, const int* y, int d,
                    int32_t* nd, double* r) {
    int m = p->m, cap = p->a_max[0];
    int z[OR_MAXD + 1];
    for (int j = 1; j <= m - 1; ++j) {
        int x = dig[m - j];
        z[j] = x + y[j] < cap ? x + y[j] : cap; /* excess rejected at delivery */
    }
    z[m] = y[m];
    int tot = 0;
    for (int j = 1; j <= m; ++j) tot += z[j];
    int cum = 0;
    int Xn[OR_MAXD + 1];
    for (int j = 1; j <= m - 1; ++j) {
        cum += z[j];
        Xn[j] = ipos(z[j + 1] - ipos(d - cum));
    }
    nd[0] = (dig[0] + 1) % p->n_periods;
    for (int j = 1; j <= m - 1; ++j) nd[m - j] = Xn[j];
    *r = -(a > 0 ? p->c_fixed : 0.0) - p->c_hold * pos((double)(tot - d)) -
         p->c_short * pos((double)(d - tot)) - p->c_waste * pos((double)(z[1] - d));
}

/* multinomial probability of y[1..m] given a and the life probabilities p_k(a) */
static double multinom_pmf(const or_mdp* p, int a, const int* y) {
    int m = p->m;
    const double* pk = p->rul_p + (size_t)a * m;
    double c = 1.0;
    int placed = 0;
    for (int k = 1; k <= m; ++k) {
        /* choose y[k] of the remaining (a - placed) */
        for (int i = 1; i <= y[k]; ++i) c = c * (double)(placed + i) / (double)i;
        placed += y[k];
        c *= pow(pk[k - 1], (double)y[k]);
    }
    return c;
}

typedef struct {
    const or_mdp* p;
    const double* V;
    const int32_t* dig;
    int a;
    const double* pd;
    double q;
} c_acc;

static void c_enum(c_acc* A, int* y, int k, int left) {
    const or_mdp* p = A->p;
    int m = p->m;
    if (k == 1) {
        y[1] = left;
        double py = multinom_pmf(p, A->a, y);
        if (py == 0.0) return;
        int32_t nd[OR_MAXD];
        for (int d = 0; d <= p->d_max[0]; ++d) {
            double pr = A->pd[d];
            if (pr == 0.0) continue;
            double r;
            trans_c(p, A->dig, A->a, y, d, nd, &r);
            A->q += py * pr * (r + p->gamma * A->V[or_encode(p, nd)]);
        }
        return;
    }
    for (int v = left; v >= 0; --v) { /* y_m first, largest first */
        y[k] = v;
        c_enum(A, y, k - 1, left - v);
    }
    (void)m;
}

static double q_c(const or_mdp* p, const double* V, const int32_t* dig, int a) {
    c_acc A;
    A.p = p;
    A.V = V;
    A.dig = dig;
    A.a = a;
    A.pd = p->pmf0 + (size_t)dig[0] * (p->d_max[0] + 1);
    A.q = 0.0;
    int y[OR_MAXD + 1];
    memset(y, 0, sizeof y);
    c_enum(&A, y, p->m, a);
    return A.q;
}

/* ------------------------------------------------------------------ backup */

static double q_sa(const or_mdp* p, const double* V, const int32_t* dig, int a) {
    if (p->family == 0) return q_a(p, V, dig, a);
    if (p->family == 1) {
        int nb = p->a_max[1] + 1;
        return q_b(p, V, dig, a / nb, a % nb);
    }
    if (p->family == 3) {
        int nb = p->a_max[1] + 1;
        return q_b1(p, V, dig, a / nb, a % nb);
    }
    return q_c(p, V, dig, a);
}

/* Q(s, .) for a list of states: q_out[i*n_actions + a]. */
int or_q_states(const or_mdp* p, const double* V, const int64_t* states, int64_t n,
                double* q_out) {
    int na = or_num_actions(p);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        int32_t dig[OR_MAXD];
        or_decode(p, states[i], dig);
        for (int a = 0; a < na; ++a) q_out[i * na + a] = q_sa(p, V, dig, a);
    }
    return 0;
}

/* max, lowest argmax and best-minus-second gap of one state's Q row */
static void best_of(const double* q, int na, double* best, int32_t* arg, double* gap) {
    double b = q[0], s = -INFINITY;
    int32_t ia = 0;
    for (int a = 1; a < na; ++a) {
        if (q[a] > b) {
            s = b;
            b = q[a];
            ia = a;
        } else if (q[a] > s) {
            s = q[a];
        }
    }
    *best = b;
    *arg = ia;
    *gap = b - s;
}

/* One synchronous sweep V -> Vnew (pi, gap optional). */
int or_sweep(const or_mdp* p, const double* V, double* Vnew, int32_t* pi, double* gap) {
    int64_t ns = or_num_states(p);
    int na = or_num_actions(p);
#pragma omp parallel
    {
        double* q = (double*)malloc(sizeof(double) * na);
#pragma omp for schedule(dynamic, 64)
        for (int64_t s = 0; s < ns; ++s) {
            int32_t dig[OR_MAXD];
            or_decode(p, s, dig);
            for (int a = 0; a < na; ++a) q[a] = q_sa(p, V, dig, a);
            double b, g;
            int32_t ia;
            best_of(q, na, &b, &ia, &g);
            Vnew[s] = b;
            if (pi) pi[s] = ia;
            if (gap) gap[s] = g;
        }
        free(q);
    }
    return 0;
}

/*
 * Value iteration from V (in: V0, out: V_ret = the last V_new).  Stops when the
 * span of V_new - V drops below thr, or after fixed_sweeps sweeps when that is
 * positive (no early stop), or at max_sweeps (returns 1).  The policy comes from
 * one more backup of V_ret.  out_stats = {sweeps, final span, max dV, min dV}.
 */
/* stop_rule 0: span rule, max(V'-V) - min(V'-V) < thr (Appendix B);
   stop_rule 1: sup-norm rule, max |V' - V| < thr (Appendix A);
   stop_rule 2: periodic rule of Appendix C with period P = n_periods: with the
   increments d_k = V_k - V_{k-1}, the paper sums gamma^-(i-j-1) d_{i-j} over the
   last P sweeps j = 0..P-1; multiplying that sum by gamma^(i-1) gives
   D(s) = sum_j gamma^j d_{i-j}(s) and the same test, which is: stop once i >= P
   and max D - min D <= 2 thr min(|max D|, |min D|). */
int or_solve(const or_mdp* p, double thr, int32_t max_sweeps, int32_t fixed_sweeps,
             int32_t stop_rule, double* V, int32_t* pi, double* gap, double* out_stats) {
    int64_t ns = or_num_states(p);
    double* Vn = (double*)malloc(sizeof(double) * ns);
    double* Vx = (double*)malloc(sizeof(double) * ns);
    const int P = p->n_periods > 0 ? p->n_periods : 1;
    double* hist = stop_rule == 2 ? (double*)malloc(sizeof(double) * ns * P) : NULL;
    int sweeps = 0, rc = 1;
    double span = INFINITY, dmax = 0.0, dmin = 0.0;
    int limit = fixed_sweeps > 0 ? fixed_sweeps : max_sweeps;
    while (sweeps < limit) {
        or_sweep(p, V, Vn, NULL, NULL);
        ++sweeps;
        dmax = -INFINITY;
        dmin = INFINITY;
        for (int64_t s = 0; s < ns; ++s) {
            double dv = Vn[s] - V[s];
            if (dv > dmax) dmax = dv;
            if (dv < dmin) dmin = dv;
        }
        span = dmax - dmin;
        int periodic_met = 0;
        if (stop_rule == 2) {
            /* increment of sweep i = sweeps kept in slot i mod P */
            double* di = hist + (size_t)(sweeps % P) * ns;
            for (int64_t s = 0; s < ns; ++s) di[s] = Vn[s] - V[s];
            if (sweeps >= P) {
                double Dmax = -INFINITY, Dmin = INFINITY;
                for (int64_t s = 0; s < ns; ++s) {
                    double D = 0.0, w = 1.0;
                    for (int j = 0; j < P; ++j) {
                        D += w * hist[(size_t)((sweeps - j) % P) * ns + s];
                        w *= p->gamma;
                    }
                    if (D > Dmax) Dmax = D;
                    if (D < Dmin) Dmin = D;
                }
                periodic_met = Dmax - Dmin <= 2.0 * thr * fmin(fabs(Dmax), fabs(Dmin));
            }
        }
        memcpy(V, Vn, sizeof(double) * ns);
        const double crit = stop_rule == 1 ? fmax(fabs(dmax), fabs(dmin)) : span;
        if (fixed_sweeps <= 0 && (stop_rule == 2 ? periodic_met : crit < thr)) {
            rc = 0;
            break;
        }
    }
    if (fixed_sweeps > 0) rc = 0;
    or_sweep(p, V, Vx, pi, gap);
    out_stats[0] = sweeps;
    out_stats[1] = span;
    out_stats[2] = dmax;
    out_stats[3] = dmin;
    free(Vn);
    free(Vx);
    free(hist);
    return rc;
}

/* Single transitions, for tests of T against an independent unit-level model.
 * omega: A {d}; B {dA, dB, k}; C {d, y_m, ..., y_1}. */
int or_transition(const or_mdp* p, int64_t s, int32_t a, const int32_t* omega,
                  int64_t* s_next, double* r) {
    int32_t dig[OR_MAXD], nd[OR_MAXD];
    or_decode(p, s, dig);
    if (p->family == 0) {
        trans_a(p, dig, a, omega[0], nd, r);
    } else if (p->family == 1) {
        int nb = p->a_max[1] + 1;
        trans_b(p, dig, a / nb, a % nb, omega[0], omega[1], omega[2], nd, r);
    } else if (p->family == 3) {
        int nb = p->a_max[1] + 1;
        trans_b1(p, dig, a / nb, a % nb, omega[0], omega[1], nd, r);
    } else {
        int y[OR_MAXD + 1];
        for (int k = 1; k <= p->m; ++k) y[k] = omega[1 + (p->m - k)];
        trans_c(p, dig, a, y, omega[0], nd, r);
    }
    *s_next = or_encode(p, nd);
    return 0;
}

/* Multinomial probability of an arrival profile (y_m..y_1) for order a (C). */
double or_arrival_prob(const or_mdp* p, int32_t a, const int32_t* y_desc) {
    int y[OR_MAXD + 1];
    for (int k = 1; k <= p->m; ++k) y[k] = y_desc[p->m - k];
    return multinom_pmf(p, a, y);
}

/* -------------------------------------------------------------- simulation */
/*
 * Rollouts of a policy (Simulation section: rollouts of warmup + horizon days from
 * a start state; the return is the discounted sum of rewards from the end of the
 * warm-up; KPIs are the service level, the wastage and the holding).
 *
 * Random numbers: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC 2011).  Draw w of block b on day t of rollout r
 * is word w of Philox(counter = {r, t, b, 0}, key = {seed, 0}), mapped to
 * u = (x >> 11) * 2^-53 in [0, 1).  Block 0 word 0 is the demand (product 0),
 * word 1 the demand of product 1 (B).  Unit i of the day (C: remaining life of
 * the i-th unit ordered; B: whether the i-th unmet customer of product 0 accepts
 * product 1) uses block 1 + i/4, word i%4.  Rollouts of different policies see the
 * same numbers.
 *
 * Sampling: the demand is the smallest d with u < CDF(d), CDF summed left to right
 * over the PMF, and d_max when there is none; a unit's remaining life is the
 * smallest k with u < p_1 + ... + p_k, and m when there is none; a customer
 * accepts substitution when u < rho.
 */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
    unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void or_philox4x64_10(const uint64_t* ctr, const uint64_t* key, uint64_t* out) {
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { /* Weyl sequence bump of the key between rounds */
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(0xD2E7470EE14C6C93ULL, x0, &hi0, &lo0);
        mulhilo64(0xCA5A826395121157ULL, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static double unif(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

/* word w of block b of day t of rollout r */
static double draw(uint64_t seed, int64_t r, int t, int b, int w) {
    uint64_t ctr[4] = {(uint64_t)r, (uint64_t)t, (uint64_t)b, 0};
    uint64_t key[2] = {seed, 0};
    uint64_t out[4];
    or_philox4x64_10(ctr, key, out);
    return unif(out[w]);
}

static int sample_pmf(const double* pmf, int dmax, double u) {
    double cdf = 0.0;
    for (int d = 0; d < dmax; ++d) {
        cdf += pmf[d];
        if (u < cdf) return d;
    }
    return dmax;
}

/* Heuristic and tabulated policies (Simulation optimization, per scenario), the
 * order written to act[0] (two products: act[0], act[1]):
 *  kind 0: table[s], split into the two products' orders for scenario B;
 *  kind 1: base stock (Scenario A): [S - I]^+, I = stock on hand and in transit;
 *  kind 2: modified base stock (Scenario B), per product k with on-hand stock I_k,
 *          oldest stock X1_k and mean demand mu_k: floor([S_k - I_k + [X1_k - mu_k]^+]^+);
 *  kind 3: (s, S) per weekday (Scenario C): [S_tau - I]^+ when I <= s_tau and
 *          s_tau < S_tau, else 0.
 * The heuristics place orders as their formulas give them, with no cap at the
 * maximum order quantity (S is the largest order a heuristic places, and the
 * paper searches S^a, S^b up to twice the maximum order quantities), except
 * Scenario C's, capped at the maximum order quantity, the range over which the
 * remaining-life distribution of an order is given.  Digits may therefore exceed
 * the state space's ranges under a heuristic; a table policy keeps them inside. */
static void policy_action(const or_mdp* p, int kind, const int32_t* table,
                          const int32_t* prm, const double* mu, const int32_t* dig,
                          int* act) {
    int nd = n_digits(p);
    int two = p->family == 1 || p->family == 3;
    if (kind == 0) {
        int a = table[or_encode(p, dig)];
        if (two) {
            act[0] = a / (p->a_max[1] + 1);
            act[1] = a % (p->a_max[1] + 1);
        } else {
            act[0] = a;
        }
        return;
    }
    if (kind == 1) {
        int I = 0;
        for (int i = 0; i < nd; ++i) I += dig[i];
        act[0] = ipos(prm[0] - I);
        return;
    }
    if (kind == 2) {
        int m = p->m;
        int w = p->family == 3 ? m : m - 1; /* digits per product */
        for (int k = 0; k < 2; ++k) {
            int I = 0;
            for (int j = 0; j < w; ++j) I += dig[k * w + j];
            int x1 = dig[k * w + (w - 1)]; /* life 1: last digit of the product */
            double v = pos((double)prm[k] - I + pos((double)x1 - mu[k]));
            act[k] = (int)floor(v);
        }
        return;
    }
    {
        int tau = dig[0], I = 0;
        for (int i = 1; i < nd; ++i) I += dig[i];
        int s_lo = prm[2 * tau], S_hi = prm[2 * tau + 1];
        int a = (s_lo < S_hi && I <= s_lo) ? ipos(S_hi - I) : 0;
        act[0] = a < p->a_max[0] ? a : p->a_max[0];
    }
}

/* the day's KPI quantities, in total and (two-product families) per product */
typedef struct {
    int64_t demand, met, expired, received, held;
    int64_t pd[2], pm[2], pe[2], pr[2], ph[2];
} or_counts;

static void or_product(or_counts* c, int k, int64_t demand, int64_t met, int64_t expired,
                       int64_t received, int64_t held) {
    c->pd[k] += demand;
    c->pm[k] += met;
    c->pe[k] += expired;
    c->pr[k] += received;
    c->ph[k] += held;
}

/* one day: sample the outcome, apply T, count the KPI quantities */
static double sim_day(const or_mdp* p, uint64_t seed, int64_t r, int t, const int32_t* dig,
                      const int* act, int32_t* nd, or_counts* c) {
    double rew;
    int m = p->m, a = act[0];
    if (p->family == 0) {
        int d = sample_pmf(p->pmf0, p->d_max[0], draw(seed, r, t, 0, 0));
        trans_a(p, dig, a, d, nd, &rew);
        int L = p->L, X[OR_MAXD + 1], tot = 0;
        for (int j = 1; j <= m; ++j) tot += (X[j] = dig[(L - 1) + (m - j)]);
        int met = d < tot ? d : tot, W;
        if (p->issuing == 1) {
            int above = tot - X[1];
            W = ipos(X[1] - ipos(d - above));
        } else {
            W = ipos(X[1] - d);
        }
        c->demand += d;
        c->met += met;
        c->expired += W;
        c->held += tot - met - W;
        c->received += nd[L - 1]; /* X_m of the next state: the units that arrived */
    } else if (p->family == 1) {
        int aA = act[0], aB = act[1];
        int dA = sample_pmf(p->pmf0, p->d_max[0], draw(seed, r, t, 0, 0));
        int dB = sample_pmf(p->pmf1, p->d_max[1], draw(seed, r, t, 0, 1));
        int sA = aA, sB = aB;
        for (int j = 0; j < m - 1; ++j) {
            sA += dig[j];
            sB += dig[(m - 1) + j];
        }
        int hA = dA < sA ? dA : sA, uA = dA - hA;
        int k = 0;
        for (int i = 0; i < uA; ++i)
            if (draw(seed, r, t, 1 + i / 4, i % 4) < p->rho) ++k;
        trans_b(p, dig, aA, aB, dA, dB, k, nd, &rew);
        int hB = dB < sB ? dB : sB, hS = k < sB - hB ? k : sB - hB;
        int keptA = 0, keptB = 0;
        for (int j = 0; j < m - 1; ++j) {
            keptA += nd[j];
            keptB += nd[(m - 1) + j];
        }
        c->demand += dA + dB;
        c->met += hA + hB + hS;
        c->received += aA + aB;
        c->held += keptA + keptB;
        c->expired += (sA - hA - keptA) + (sB - hB - hS - keptB);
        /* product 0's customers served by product 1 count as met for product 0 */
        or_product(c, 0, dA, hA + hS, sA - hA - keptA, aA, keptA);
        or_product(c, 1, dB, hB, sB - hB - hS - keptB, aB, keptB);
    } else if (p->family == 3) {
        int aA = act[0], aB = act[1];
        int dA = sample_pmf(p->pmf0, p->d_max[0], draw(seed, r, t, 0, 0));
        int dB = sample_pmf(p->pmf1, p->d_max[1], draw(seed, r, t, 0, 1));
        int Ia = 0, Ib = 0;
        for (int j = 0; j < m; ++j) {
            Ia += dig[j];
            Ib += dig[m + j];
        }
        int hB = dB < Ib ? dB : Ib, excess = dB - hB, du = 0;
        for (int i = 0; i < excess; ++i)
            if (draw(seed, r, t, 1 + i / 4, i % 4) < p->rho) ++du;
        int hA = dA + du < Ia ? dA + du : Ia;
        trans_b1(p, dig, aA, aB, hA, hB, nd, &rew);
        int keptA = 0, keptB = 0;
        for (int j = 1; j < m; ++j) {
            keptA += nd[j];
            keptB += nd[m + j];
        }
        c->demand += dA + dB;
        c->met += hA + hB; /* product b's demand met by product a counts as met */
        c->received += aA + aB;
        c->held += keptA + keptB;
        c->expired += (Ia - hA - keptA) + (Ib - hB - keptB);
        /* of product a's issues, its own customers took min(dA, Ia) (they come
         * first); the rest went to product b's customers */
        int ownA = dA < Ia ? dA : Ia;
        or_product(c, 0, dA, ownA, Ia - hA - keptA, aA, keptA);
        or_product(c, 1, dB, hB + (hA - ownA), Ib - hB - keptB, aB, keptB);
    } else {
        int d = sample_pmf(p->pmf0 + (size_t)dig[0] * (p->d_max[0] + 1), p->d_max[0],
                           draw(seed, r, t, 0, 0));
        int y[OR_MAXD + 1];
        for (int k = 1; k <= m; ++k) y[k] = 0;
        const double* pk = p->rul_p + (size_t)a * m;
        for (int i = 0; i < a; ++i) {
            double u = draw(seed, r, t, 1 + i / 4, i % 4), cum = 0.0;
            int life = m;
            for (int k = 1; k < m; ++k) {
                cum += pk[k - 1];
                if (u < cum) {
                    life = k;
                    break;
                }
            }
            y[life]++;
        }
        trans_c(p, dig, a, y, d, nd, &rew);
        int cap = p->a_max[0], tot = 0, before = 0, z1 = 0;
        for (int j = 1; j <= m - 1; ++j) {
            int x = dig[m - j], z = x + y[j] < cap ? x + y[j] : cap;
            if (j == 1) z1 = z;
            tot += z;
            before += x;
        }
        tot += y[m];
        c->demand += d;
        c->met += d < tot ? d : tot;
        c->expired += ipos(z1 - d);
        c->held += ipos(tot - d); /* includes the units that expire tonight */
        c->received += tot - before;
    }
    return rew;
}

/* n_pol policies (params: [n_pol][16]) x n_roll rollouts each.
 * ret[p*n_roll + r] = sum_{t=warmup}^{warmup+horizon-1} gamma^(t-warmup) R_t;
 * kpi[(p*n_roll + r)*3 + 0..2] = service level % (met/demand, 100 when no demand),
 * wastage % (expired/received, 0 when nothing arrived), mean holding per day; all
 * counted over the horizon days only.  pkpi (NULL to skip; two-product families)
 * [(p*n_roll + r)*2 + k][3]: the same three KPIs of product k alone, the demand of
 * the product whose customers substitute counting as met when the other product
 * serves it (Appendix B, KPI tables). */
static void or_kpis(double* out, int64_t demand, int64_t met, int64_t expired,
                    int64_t received, int64_t held, int32_t horizon) {
    out[0] = demand > 0 ? 100.0 * (double)met / (double)demand : 100.0;
    out[1] = received > 0 ? 100.0 * (double)expired / (double)received : 0.0;
    out[2] = horizon > 0 ? (double)held / (double)horizon : 0.0;
}

int or_simulate(const or_mdp* p, int32_t kind, const int32_t* table, const int32_t* params,
                const double* mu, int32_t n_pol, int32_t n_roll, int32_t warmup,
                int32_t horizon, uint64_t seed, int64_t start, double* ret, double* kpi,
                double* pkpi) {
    int64_t total = (int64_t)n_pol * n_roll;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < total; ++i) {
        int pol = (int)(i / n_roll);
        int64_t r = i % n_roll;
        const int32_t* prm = params ? params + (size_t)pol * 16 : NULL;
        int32_t dig[OR_MAXD], nd[OR_MAXD];
        int nd_count = n_digits(p);
        double g = 1.0, acc = 0.0;
        or_decode(p, start, dig);
        or_counts c;
        memset(&c, 0, sizeof c);
        for (int t = 0; t < warmup + horizon; ++t) {
            int act[2] = {0, 0};
            policy_action(p, kind, table, prm, mu, dig, act);
            or_counts day;
            memset(&day, 0, sizeof day);
            double rew = sim_day(p, seed, r, t, dig, act, nd, &day);
            if (t >= warmup) {
                acc += g * rew;
                g *= p->gamma;
                c.demand += day.demand;
                c.met += day.met;
                c.expired += day.expired;
                c.received += day.received;
                c.held += day.held;
                for (int k = 0; k < 2; ++k)
                    or_product(&c, k, day.pd[k], day.pm[k], day.pe[k], day.pr[k], day.ph[k]);
            }
            memcpy(dig, nd, sizeof(int32_t) * nd_count); /* the state is kept as digits */
        }
        ret[i] = acc;
        or_kpis(kpi + 3 * i, c.demand, c.met, c.expired, c.received, c.held, horizon);
        if (pkpi)
            for (int k = 0; k < 2; ++k)
                or_kpis(pkpi + (2 * i + k) * 3, c.pd[k], c.pm[k], c.pe[k], c.pr[k], c.ph[k],
                        horizon);
    }
    return 0;
}
