// Descriptor validation, host tables and the small accessors of the C ABI.
#include "mdp.h"

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdlib>
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

static int64_t ipow_i(int64_t b, int e) {
    int64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

// Scenario A expected one-day reward without the order cost, as a table over
// (X_1, total stock) for FIFO or (X_1, X_2 + ... + X_m) for LIFO:
// sum_d P(d) (-C_h [X - d - W]^+ - C_s [d - X]^+ - C_w W) with W from the FIFO or
// LIFO issuing equation (Appendix A, reward equation).
// Work list of the scenario-A backup kernel for G tiles per wavefront (0: the rule
// below) and CH path points per staged chunk (0: as many as the staging lanes allow).
// One wavefront takes G tiles of equal digit sum b (so their loops run in lockstep),
// R lanes each.  Tiles are grouped per block of G in-transit vectors and, inside one
// digit sum, by (X_m..X_3) then in-transit vector, so a full group is one (X_m..X_3)
// over G in-transit vectors.  The rule: G = floor(64 / R), or 2 when full groups
// would give fewer wavefronts than the chip has SIMDs (1,024): more wavefronts, and
// each stages longer chunks of its path.  The autotuner (families.cpp) times other
// choices at the first solve of a shape.  Results do not depend on G or CH (each
// lane's arithmetic is its own tile's).  PVI_A_GROUP=<G> (1 .. floor(64 / R)) and
// PVI_A_CHUNK=<CH> fix them, for tests.
void build_a_work_list(pvi_mdp* p, int G_req, int CH_req) {
    const int R = p->rad[0];
    int64_t nh = 1;
    for (int i = 0; i < p->L - 1; ++i) nh *= R;
    const int64_t nzt = p->m >= 2 ? (int64_t)ipow_i(R, p->m - 2) : 1;
    const int gmax = a_group_max(p);
    p->a_G = G_req > 0 ? std::min(G_req, gmax)
                       : (nh * nzt / gmax < 1024 ? std::min(gmax, 2) : gmax);
    if (const char* force = std::getenv("PVI_A_GROUP")) {
        const int g = std::atoi(force);
        if (g >= 1 && g <= gmax) p->a_G = g;
    }
    const int G = p->a_G;
    const int chmax = a_chunk_max(p, G);
    p->a_CH = CH_req > 0 ? std::min(CH_req, chmax) : chmax;
    if (const char* force = std::getenv("PVI_A_CHUNK")) {
        const int c = std::atoi(force);
        if (c >= 1 && c <= chmax) p->a_CH = c;
    }
    std::vector<int> zsum(nzt, 0);
    for (int64_t z = 0; z < nzt; ++z) {
        int64_t t = z;
        for (int i = 2; i <= p->m - 1; ++i) {
            zsum[z] += (int)(t % R);
            t /= R;
        }
    }
    const int bmax = std::max(0, p->m - 2) * (R - 1);
    p->a_groups.clear();
    for (int64_t hb = 0; hb < nh; hb += G) {
        const int64_t he = std::min<int64_t>(hb + G, nh);
        for (int b = bmax; b >= 0; --b) {
            int fill = 0;
            for (int64_t z = 0; z < nzt; ++z) {
                if (zsum[z] != b) continue;
                for (int64_t h = hb; h < he; ++h) {
                    p->a_groups.push_back((int32_t)(h * nzt + z));
                    if (++fill == G) fill = 0;
                }
            }
            for (; fill != 0 && fill < G; ++fill) p->a_groups.push_back(-1);
        }
    }
    // Workgroups are dispatched round-robin over the 8 XCDs and the kernel gives
    // XCD x a contiguous range of groups (its L2 then holds the V blocks of those
    // in-transit vectors).  Sorting each range by digit sum, longest path first,
    // makes the in-order dispatch onto freed slots a longest-first list schedule,
    // which shortens the tail of the launch.
    const int ng = (int)(p->a_groups.size() / G), q = ng >> 3, r = ng & 7;
    std::vector<int32_t> sorted;
    sorted.reserve(p->a_groups.size());
    for (int x = 0; x < 8; ++x) {
        const int lo = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
        const int cnt = q + (x < r ? 1 : 0);
        std::vector<int> idx(cnt);
        for (int k = 0; k < cnt; ++k) idx[k] = lo + k;
        auto bsum = [&](int grp) { return zsum[p->a_groups[(size_t)grp * G] % nzt]; };
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return bsum(a) > bsum(b); });
        for (int k : idx)
            sorted.insert(sorted.end(), p->a_groups.begin() + (size_t)k * G,
                          p->a_groups.begin() + (size_t)(k + 1) * G);
    }
    p->a_groups.swap(sorted);
}

int a_group_max(const pvi_mdp* p) { return std::min(16, std::max(1, 64 / p->rad[0])); }

// The kernel pads the actions to RMAX = 8, 16, 24 or 32 and stages each path point
// with RMAX / 8 lanes of 8 actions: CH points per chunk of G tiles fill <= 64 lanes.
int a_chunk_max(const pvi_mdp* p, int G) {
    const int R = p->rad[0];
    const int rmax = R <= 8 ? 8 : R <= 16 ? 16 : R <= 24 ? 24 : 32;
    return std::max(1, 64 / ((rmax / 8) * G));
}

static void build_a_tables(pvi_mdp* p) {
    const int R = p->rad[0], dm = p->dmax[0];
    const auto& P = p->pmf[0];
    // the kernel reads P, F and G at up to 2R + (path length):
    // pad with P = 0, F = 1, G = 0 beyond d_max
    const int lp_max = (p->m >= 2 ? (p->m - 2) * (R - 1) : 0) + (p->m >= 2 ? R : 1);
    p->tab = std::max(dm + 10, 2 * R + 8 + lp_max);
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
    // with one life class LIFO and FIFO coincide and the FIFO kernel and table serve
    const bool lifo = p->d.issuing == PVI_LIFO && p->m >= 2;
    // FIFO: r0[X_1][X], X the total stock; LIFO: r0[X_1][K], K = X_2 + ... + X_m,
    // whose waste is what the demand leaves of X_1 after the younger units
    for (int x1 = 0; x1 < R; ++x1)
        for (int k = 0; k < p->xt; ++k) {
            const int X = lifo ? x1 + k : k;
            double e = 0.0;
            for (int d = 0; d <= dm; ++d) {
                const int W = lifo ? std::max(x1 - std::max(d - k, 0), 0) : std::max(x1 - d, 0);
                const double r = -ch * std::max(X - d - W, 0) - cs * std::max(d - X, 0) - cw * W;
                e += P[d] * r;
            }
            p->a_r0[(size_t)x1 * p->xt + k] = e;
        }
    // multiply-adds that contribute to a result, per sweep, in the per-diagonal
    // prefix-sum scheme: for a tile of digit sum b (of X_m..X_3) and one action,
    // every live diagonal u in [max(b,1), b + r2 + R - 2] accumulates once per path
    // point (N = 0 .. b + r2 - 2, the first being the G(u) S[0] start), and every
    // one of the r2 * R states adds F(X_1) S[N] once
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
        const int nmin = std::max((int)b, 1), nmax = (int)b + r2 - 1;
        const int64_t live = std::max(0, nmax + R - 1 - nmin + 1);
        const int64_t per = (nmax >= 1 ? live * nmax : 0) + (int64_t)r2 * R;
        ex += cnt[b] * per;
    }
    p->executed_per_sweep = nh * ex * R;
    if (lifo) {
        // per tile and action: K + 1 terms for each X_m = t (K = b + t)
        int64_t ex2 = 0;
        for (size_t b = 0; b < cnt.size(); ++b)
            for (int t = 0; t < R; ++t) ex2 += cnt[b] * ((int64_t)b + t + 1);
        p->executed_per_sweep = nh * ex2 * R;
    }

    build_a_work_list(p, 0, 0);
    p->logical_per_sweep = p->ns * p->na * (int64_t)(dm + 1);
}

// Scenario B tables (Appendix B reward equation; substitution of the Scenario B
// description): product-1 demand including substitutes given product-0 unmet
// demand u, E[u][e] = sum_k Bin(k; u, rho) P1(e - k), and expected revenues.
static void build_b_tables(pvi_mdp* p) {
    const int d0 = p->dmax[0], d1 = p->dmax[1], m = p->m;
    const int R0 = p->rad[0], R1 = p->rad[1];
    const auto& P0 = p->pmf[0];
    const auto& P1 = p->pmf[1];
    const int na = (int)std::pow(R0, m - 1), nb = (int)std::pow(R1, m - 1);
    p->b_rows = na + d0;
    p->b_emax = d0 + d1;
    p->b_ew = p->b_emax + 1;
    p->b_sw = m * (R1 - 1) + 1;
    p->b_rexp0.assign((size_t)m * (R0 - 1) + 1, 0.0);
    for (size_t s0 = 0; s0 < p->b_rexp0.size(); ++s0) {
        double e = 0.0;
        for (int d = 0; d <= d0; ++d) e += P0[d] * std::min<double>(d, (double)s0);
        p->b_rexp0[s0] = p->d.c_rev[0] * e;
    }
    const size_t ew = p->b_ew;
    p->b_epmf.assign((size_t)(d0 + 1) * ew, 0.0);
    p->b_ecdf.assign((size_t)(d0 + 1) * ew, 1.0);
    p->b_etail.assign((size_t)(d0 + 1) * ew, 0.0);
    p->b_rexp1.assign((size_t)(d0 + 1) * p->b_sw, 0.0);
    for (int u = 0; u <= d0; ++u) {
        double* E = p->b_epmf.data() + u * ew;
        for (int k = 0; k <= u; ++k) {
            const double bk = binom_pmf(k, u, p->d.subst_rho);
            if (bk == 0.0) continue;
            for (int d = 0; d <= d1; ++d) E[d + k] += bk * P1[d];
        }
        double c = 0.0;
        for (size_t e = 0; e < ew; ++e) {
            c += E[e];
            p->b_ecdf[u * ew + e] = e + 1 == ew ? 1.0 : c;
        }
        double t = 0.0;
        for (int e = (int)ew - 1; e >= 0; --e) {
            t += E[e];
            p->b_etail[u * ew + e] = t;
        }
        for (int s1 = 0; s1 < p->b_sw; ++s1) {
            double r = 0.0;
            for (size_t e = 0; e < ew; ++e) r += E[e] * std::min<double>((double)e, s1);
            p->b_rexp1[(size_t)u * p->b_sw + s1] = p->d.c_rev[1] * r;
        }
    }
    // the tiled sweep kernels keep one accumulator per oldest digit (at most 16 per
    // product) and every product-0 demand value in registers (at most PVI_B_JMAX)
    const char* tiled = std::getenv("PVI_B_TILED");
    p->b_tiled = !(tiled && std::strcmp(tiled, "0") == 0) && m >= 2 && R0 <= 16 &&
                 R1 <= PVI_B_R1MAX && d0 + 1 <= PVI_B_JMAX &&
                 (double)p->b_rows * std::pow((double)R1, m) < 2147483647.0;
    if (p->b_tiled) {
        // x1 + k for x1 < 16 and k up to the (m - 1)(R1 - 1) younger units, or up to
        // the 32 points the stage-1 kernel unrolls
        p->b_ewp = (int)ew + 16 + std::max((m - 1) * (R1 - 1), 32);
        p->b_ppad.assign((size_t)(d0 + 1) * p->b_ewp, 0.0);
        p->b_gpad.assign((size_t)(d0 + 1) * p->b_ewp, 0.0);
        for (int u = 0; u <= d0; ++u)
            for (size_t e = 0; e < ew; ++e) {
                p->b_ppad[(size_t)u * p->b_ewp + e] = p->b_epmf[u * ew + e];
                p->b_gpad[(size_t)u * p->b_ewp + e] = p->b_etail[u * ew + e];
            }
    }
    // stage 1: sum over the FIFO path of each (row, product-1 part); stage 2: d0 terms
    int64_t ex1 = 0;
    for (int ib = 0; ib < nb; ++ib)
        for (int a1 = 0; a1 < R1; ++a1) {
            int rest = ib, x1 = rest % R1, K = a1;
            rest /= R1;
            for (int j = 1; j <= m - 2; ++j) {
                K += rest % R1;
                rest /= R1;
            }
            for (int u = 0; u <= d0; ++u) {
                const int emax = d1 + u;
                const int kmax = K == 0 ? 0 : std::max(0, std::min(K, emax - x1));
                ex1 += (int64_t)(kmax + 1) * (u == 0 ? na : 1);
            }
        }
    p->executed_per_sweep = ex1 + p->ns * p->na * (int64_t)(d0 + 1);
    p->logical_per_sweep = p->ns * p->na * (int64_t)(d0 + 1) * (d1 + 1);
}

// Scenario C tables (Appendix C): per-weekday demand with padding, the expected
// one-day reward of a post-arrival stock vector z (holding counts the units that
// expire, as the reward equation writes it), and the binomial factors of the
// remaining-life multinomial.
static void build_c_tables(pvi_mdp* p) {
    const int R = p->rad[0], m = p->m, P = p->P, dm = p->dmax[0];
    p->c_exogenous = true;
    for (int k = 2; k <= m; ++k)
        if (p->d.rul_c1[k - 1] != 0.0) p->c_exogenous = false;
    p->c_lpmax = (m - 2) * (R - 1) + R;
    p->c_tab = std::max(dm + 10, R + 8 + p->c_lpmax);
    const int tab = p->c_tab;
    p->c_pmf.assign((size_t)P * tab, 0.0);
    p->c_cdf.assign((size_t)P * tab, 1.0);
    p->c_tail.assign((size_t)P * tab, 0.0);
    p->c_xt = m * (R - 1) + 1;
    p->c_r0.assign((size_t)P * R * p->c_xt, 0.0);
    const double ch = p->d.c_hold, cs = p->d.c_short, cw = p->d.c_waste;
    for (int t = 0; t < P; ++t) {
        const double* Pd = p->pmf[0].data() + (size_t)t * (dm + 1);
        double c = 0.0;
        for (int d = 0; d <= dm; ++d) {
            p->c_pmf[(size_t)t * tab + d] = Pd[d];
            c += Pd[d];
            p->c_cdf[(size_t)t * tab + d] = d == dm ? 1.0 : c;
        }
        double tl = 0.0;
        for (int d = dm; d >= 0; --d) {
            tl += Pd[d];
            p->c_tail[(size_t)t * tab + d] = tl;
        }
        for (int z1 = 0; z1 < R; ++z1)
            for (int Z = z1; Z < p->c_xt; ++Z) {
                double e = 0.0;
                for (int d = 0; d <= dm; ++d)
                    e += Pd[d] * (-ch * std::max(Z - d, 0) - cs * std::max(d - Z, 0) -
                                  cw * std::max(z1 - d, 0));
                p->c_r0[((size_t)t * R + z1) * p->c_xt + Z] = e;
            }
    }
    // Binomial factors of the remaining-life multinomial.  Exogenous: one set
    // [m][R][R] from p_k(0).  Order-dependent: one set per order a, [a][m][R][R],
    // from p_k(a).  Row a of binm always uses p_m(a).
    const int nsets = p->c_exogenous ? 1 : R;
    p->c_binq.assign((size_t)nsets * m * R * R, 0.0);
    for (int a = 0; a < nsets; ++a) {
        const double* pk = p->life.data() + (size_t)a * m;
        double* bq = p->c_binq.data() + (size_t)a * m * R * R;
        double cum = pk[0];
        for (int j = 2; j <= m - 1; ++j) {
            cum += pk[j - 1];
            const double q = cum > 0.0 ? pk[j - 1] / cum : 0.0;
            for (int r = 0; r < R; ++r)
                for (int y = 0; y <= r; ++y) bq[((size_t)j * R + r) * R + y] = binom_pmf(y, r, q);
        }
    }
    p->c_binm.assign((size_t)R * R, 0.0);
    for (int a = 0; a < R; ++a) {
        const double pm = p->life[(size_t)(p->c_exogenous ? 0 : a) * m + (m - 1)];
        for (int y = 0; y <= a; ++y) p->c_binm[(size_t)a * R + y] = binom_pmf(y, a, pm);
    }
    p->c_pair_y.clear();
    p->c_pair_r.clear();
    p->c_pair_base.assign(R, 0);
    for (int y = 0; y < R; ++y) {
        p->c_pair_base[y] = (int32_t)p->c_pair_y.size();
        for (int r = 0; r + y < R; ++r) {
            p->c_pair_y.push_back(y);
            p->c_pair_r.push_back(r);
        }
    }
    p->c_npair = (int)p->c_pair_y.size();
    // multiply-adds per sweep: U (FIFO path), each merge, and the final order sum
    const int64_t nblk = p->ns / P;
    int64_t nzu = 1;
    for (int i = 0; i < m - 2; ++i) nzu *= R;
    std::vector<int64_t> cnt(1, 1);
    for (int i = 0; i < m - 2; ++i) {
        std::vector<int64_t> nx(cnt.size() + R - 1, 0);
        for (size_t b = 0; b < cnt.size(); ++b)
            for (int v = 0; v < R; ++v) nx[b + v] += cnt[b];
        cnt.swap(nx);
    }
    int64_t exu = 0;
    for (size_t b = 0; b < cnt.size(); ++b)
        for (int z2 = 0; z2 < R; ++z2)
            for (int z1 = 0; z1 < R; ++z1) {
                const int N = (int)b + z2;
                exu += cnt[b] * ((N == 0 ? 0 : std::max(0, std::min(N, dm - z1))) + 1);
            }
    int64_t merge_terms = 0;  // over all merge levels, per state block
    if (p->c_exogenous) {
        for (int i = 0; i < p->c_npair; ++i) merge_terms += (int64_t)(m - 2) * (p->c_pair_r[i] + 1);
    } else if (m >= 3) {
        // per order a: rows y_m + r <= a at the lower levels, r = a - y_m at the top
        for (int a = 0; a < R; ++a)
            for (int ym = 0; ym <= a; ++ym) {
                for (int r = 0; r <= a - ym; ++r) merge_terms += (int64_t)(m - 3) * (r + 1);
                merge_terms += a - ym + 1;
            }
    }
    const int64_t final_terms = (int64_t)R * (R + 1) / 2;
    p->executed_per_sweep = P * (exu + merge_terms * nblk + final_terms * nblk);
    // logical: every (d, y) outcome of every (state, order): (d_max+1) C(a+m-1, m-1)
    int64_t comps = 0;
    for (int a = 0; a < R; ++a) {
        int64_t c = 1;  // C(a+m-1, m-1)
        for (int i = 1; i <= m - 1; ++i) c = c * (a + i) / i;
        comps += c;
    }
    p->logical_per_sweep = p->ns * comps * (dm + 1);
}

// Scenario B as the paper runs it (Scenario B description, Appendix B).  With I_a,
// I_b the stock of each product, the issued units (h_a, h_b) have
//   P(h_a, h_b) = [h_b < I_b] P(D_b = h_b) PA[I_a][h_a] + [h_b = I_b] J[I_b][I_a][h_a]
// where PA is the demand of a capped at I_a and J is the joint probability that b
// runs out and a issues h_a: sum over D_b = I_b + c of P(D_b) P(min(D_a + Bin(c, rho),
// I_a) = h_a).  The cumulative form JC serves the first point of the FIFO path; the
// kernels weight a's own demand from the 1-D tables P(D_a = h), P(D_a <= h), P(D_a >= h).
static void build_b1_tables(pvi_mdp* p) {
    const int m = p->m, HA = m * (p->rad[0] - 1) + 1, HB = m * (p->rad[1] - 1) + 1;
    const double rho = p->d.subst_rho;
    const std::vector<double>& pa = p->pmf[0];  // [d_max0 + 1]
    const std::vector<double>& pb = p->pmf[1];
    const int da = p->dmax[0], db = p->dmax[1];
    p->b1_ha = HA;
    p->b1_hb = HB;
    auto capped_row = [&](const std::vector<double>& dist, int I, double* out) {
        double rest = 0.0;
        for (int h = 0; h <= I; ++h) out[h] = 0.0;
        for (size_t t = 0; t < dist.size(); ++t) {
            if ((int)t < I) out[t] += dist[t];
            else rest += dist[t];
        }
        out[I] += rest;
    };
    p->b1_pa.assign((size_t)HA * HA, 0.0);
    for (int Ia = 0; Ia < HA; ++Ia) capped_row(pa, Ia, &p->b1_pa[(size_t)Ia * HA]);
    p->b1_pa1.assign(HA + 1, 0.0);
    p->b1_fa.assign(HA + 1, 1.0);
    p->b1_ga.assign(HA + 1, 0.0);
    {
        double c = 0.0;
        for (int h = 0; h <= HA; ++h) {
            const double v = h <= da ? pa[h] : 0.0;
            p->b1_pa1[h] = v;
            c += v;
            p->b1_fa[h] = h >= da ? 1.0 : c;
        }
        double t = 0.0;
        for (int h = da; h >= 0; --h) {
            t += pa[h];
            if (h <= HA) p->b1_ga[h] = t;
        }
    }
    p->b1_pb.assign(HB + 1, 0.0);
    p->b1_fb.assign(HB + 1, 1.0);
    {
        double c = 0.0;
        for (int h = 0; h <= HB; ++h) {
            const double v = h <= db ? pb[h] : 0.0;
            p->b1_pb[h] = v;
            c += v;
            p->b1_fb[h] = h >= db ? 1.0 : c;
        }
    }
    // distribution of D_a plus the accepted substitutes of c unmet customers of b
    std::vector<std::vector<double>> plus(db + 1);
    for (int c = 0; c <= db; ++c) {
        std::vector<double>& v = plus[c];
        v.assign(da + c + 1, 0.0);
        for (int u = 0; u <= c; ++u) {
            const double pu = binom_pmf(u, c, rho);
            if (pu == 0.0) continue;
            for (int d = 0; d <= da; ++d) v[d + u] += pa[d] * pu;
        }
    }
    p->b1_j.assign((size_t)HB * HA * HA, 0.0);
    p->b1_jc.assign((size_t)HB * HA * HA, 0.0);
    std::vector<double> acc(da + db + 1), row(HA);
    for (int Ib = 0; Ib < HB; ++Ib) {
        std::fill(acc.begin(), acc.end(), 0.0);
        for (int d = Ib; d <= db; ++d) {
            const std::vector<double>& v = plus[d - Ib];
            for (size_t t = 0; t < v.size(); ++t) acc[t] += pb[d] * v[t];
        }
        for (int Ia = 0; Ia < HA; ++Ia) {
            capped_row(acc, Ia, row.data());
            double c = 0.0;
            for (int h = 0; h < HA; ++h) {
                const double v = h <= Ia ? row[h] : 0.0;
                p->b1_j[((size_t)Ib * HA + Ia) * HA + h] = v;
                p->b1_jc[((size_t)Ib * HA + Ia) * HA + h] = c += v;
            }
        }
    }
    // expected one-day revenue per (I_a, I_b): the reward without the order cost,
    // and the initial values of the solve
    p->b1_rev.assign((size_t)HA * HB, 0.0);
    const double ra = p->d.c_rev[0], rb = p->d.c_rev[1];
    for (int Ia = 0; Ia < HA; ++Ia)
        for (int Ib = 0; Ib < HB; ++Ib) {
            double e = 0.0;
            for (int hb = 0; hb < Ib; ++hb)
                for (int ha = 0; ha <= Ia; ++ha)
                    e += p->b1_pb[hb] * p->b1_pa[(size_t)Ia * HA + ha] * (ra * ha + rb * hb);
            for (int ha = 0; ha <= Ia; ++ha)
                e += p->b1_j[((size_t)Ib * HA + Ia) * HA + ha] * (ra * ha + rb * Ib);
            p->b1_rev[(size_t)Ia * HB + Ib] = e;
        }
    // multiply-adds per sweep: stage W (one per B path point below I_b), stage Y (one
    // per A path point per I_b), the final sum (one per A path point per action, plus Y)
    const int64_t NA = p->ns / ipow_i(p->rad[1], m), NB = ipow_i(p->rad[1], m);
    int64_t pts_a = 0, pts_b = 0;  // path points summed over all stock vectors
    for (int64_t x = 0; x < NA; ++x) {
        int64_t v = x;
        int sum = 0, x1 = (int)(v % p->rad[0]);
        for (int i = 0; i < m; ++i, v /= p->rad[0]) sum += (int)(v % p->rad[0]);
        pts_a += sum - x1 + 1;
    }
    for (int64_t x = 0; x < NB; ++x) {
        int64_t v = x;
        int sum = 0, x1 = (int)(v % p->rad[1]);
        for (int i = 0; i < m; ++i, v /= p->rad[1]) sum += (int)(v % p->rad[1]);
        pts_b += sum > 0 ? std::max(sum - x1, 1) : 0;
    }
    const int64_t na1 = NA / p->rad[0];
    p->executed_per_sweep = (int64_t)p->na * (na1 * pts_b + HB * pts_a + NB * (pts_a + NA));
    p->logical_per_sweep = p->ns * p->na * (int64_t)HA * HB;
}

}  // namespace pvi

using namespace pvi;

extern "C" {

const char* pvi_last_error(void) { return pvi::g_err.c_str(); }

pvi_status mdp_create(const pvi_mdp_desc* desc, pvi_mdp** out) {
    if (!desc || !out) return fail(PVI_E_INVALID, "mdp_create: NULL argument");
    // callers built against the layout that ended at `gamma` are accepted; fields
    // past their struct_size read as zero
    if (desc->struct_size < offsetof(pvi_mdp_desc, issuing))
        return fail(PVI_E_INVALID, "mdp_create: struct_size too small");
    pvi_mdp_desc dc{};
    std::memcpy(&dc, desc, std::min<size_t>(desc->struct_size, sizeof(pvi_mdp_desc)));
    dc.struct_size = sizeof(pvi_mdp_desc);
    const pvi_mdp_desc& d = dc;
    if (d.issuing != PVI_FIFO && d.issuing != PVI_LIFO)
        return fail(PVI_E_INVALID, "mdp_create: issuing must be PVI_FIFO or PVI_LIFO");
    if (d.issuing == PVI_LIFO && d.family != PVI_FAMILY_LEADTIME)
        return fail(PVI_E_INVALID, "mdp_create: LIFO issuing is defined for scenario A only");
    if (d.family < 0 || d.family > 3) return fail(PVI_E_INVALID, "mdp_create: bad family");
    if (d.m < 1 || d.m > PVI_MAX_LIFE) return fail(PVI_E_INVALID, "mdp_create: m out of range");
    const bool b1 = d.family == PVI_FAMILY_SUBST2_L1;
    if (!(d.gamma > 0.0 && (d.gamma < 1.0 || (b1 && d.gamma == 1.0))))
        return fail(PVI_E_INVALID, b1 ? "mdp_create: gamma must be in (0, 1]"
                                      : "mdp_create: gamma must be in (0, 1)");
    const double costs[] = {d.c_var[0], d.c_var[1], d.c_fixed, d.c_hold, d.c_short,
                            d.c_waste, d.c_rev[0], d.c_rev[1], d.subst_rho};
    for (double c : costs)
        if (!is_finite(c)) return fail(PVI_E_INVALID, "mdp_create: non-finite cost");
    const int nprod = (d.family == PVI_FAMILY_SUBST2 || b1) ? 2 : 1;
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
    } else if (b1) {
        if (d.lead_time != 1)
            return fail(PVI_E_INVALID, "mdp_create: the lead-time-1 two-product family needs L = 1");
        if (2 * d.m > 16) return fail(PVI_E_INVALID, "mdp_create: too many state digits");
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
    if ((d.family == PVI_FAMILY_SUBST2 || b1) && !(d.subst_rho >= 0.0 && d.subst_rho <= 1.0))
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
    } else if (b1) {
        p->ndig = 2 * d.m;
        for (int i = 0; i < d.m; ++i) {
            p->radix[i] = p->rad[0];
            p->radix[d.m + i] = p->rad[1];
        }
    } else {
        p->ndig = d.m;
        p->radix[0] = P;
        for (int i = 1; i < d.m; ++i) p->radix[i] = p->rad[0];
    }
    // scenario C builds no host table that grows with the states, so it accepts up
    // to 2^40 of them; beyond 2^31 its handle serves heuristic rollouts only
    const int64_t cap = d.family == PVI_FAMILY_RUL_WEEKDAY ? (int64_t(1) << 40)
                                                           : (int64_t(1) << 31);
    p->ns = 1;
    for (int i = 0; i < p->ndig; ++i) {
        p->ns *= p->radix[i];
        if (p->ns > cap) {
            delete p;
            return fail(PVI_E_INVALID, d.family == PVI_FAMILY_RUL_WEEKDAY
                                           ? "mdp_create: more than 2^40 states"
                                           : "mdp_create: more than 2^31 states");
        }
    }
    p->na = nprod == 2 ? p->rad[0] * p->rad[1] : p->rad[0];
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
    if (d.family == PVI_FAMILY_SUBST2 && d.m >= 2) build_b_tables(p);
    if (d.family == PVI_FAMILY_RUL_WEEKDAY) build_c_tables(p);
    if (b1) build_b1_tables(p);
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
    const int nprod =
        (p->family == PVI_FAMILY_SUBST2 || p->family == PVI_FAMILY_SUBST2_L1) ? 2 : 1;
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
