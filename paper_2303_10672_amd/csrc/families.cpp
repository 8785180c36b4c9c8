// Per-family dispatch: kernel parameter blocks and launches.
#include "families.h"

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

namespace pvi {

static int64_t ipow(int64_t b, int e) {
    int64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

ADev make_adev(const pvi_mdp* p) {
    ADev a{};
    const int R = p->rad[0];
    a.R = R;
    a.m = p->m;
    a.dmax = p->dmax[0];
    a.xt = p->xt;
    a.tab = p->tab;
    a.nz = p->m >= 2 ? (int)ipow(R, p->m - 2) : 1;
    a.r2 = p->m >= 2 ? R : 1;
    a.tiles = (int)(ipow(R, p->L - 1) * a.nz);
    // LIFO (m >= 2) has its own kernel over tiles (O, X_{m-1}..X_2); with one life
    // class the two issuing orders coincide and the FIFO kernel runs
    a.lifo = (p->d.issuing == PVI_LIFO && p->m >= 2) ? 1 : 0;
    a.lmax = (p->m >= 2 ? (p->m - 2) * (R - 1) : 0) + a.r2;
    a.G = p->a_G;
    a.CH = p->a_CH;
    a.groups = p->dev.agroups;
    a.ngroups = p->a_G > 0 ? (int)(p->a_groups.size() / p->a_G) : 0;
    a.stride_a = ipow(R, p->m + p->L - 2);
    a.stride_h = ipow(R, p->m - 1);
    for (int i = 0; i < 8; ++i) a.pow_y[i] = (int)ipow(R, i);
    a.gamma = p->d.gamma;
    a.cvar = p->d.c_var[0];
    a.pmf = p->dev.pmf;
    a.cdf = p->dev.cdf;
    a.tail = p->dev.tail;
    a.r0 = p->dev.r0;
    a.ctl = p->dev.ctl;
    a.partials = p->dev.partials;
    a.pi = p->dev.pi;
    a.gap = p->dev.gap;
    return a;
}

static BDev make_bdev(const pvi_mdp* p) {
    BDev b{};
    b.m = p->m;
    b.r0 = p->rad[0];
    b.r1 = p->rad[1];
    b.r1pad = PVI_B_R1MAX + 2;  // row stride of the LDS Z block: 16-byte rows, fewer bank conflicts
    b.na = (int)ipow(p->rad[0], p->m - 1);
    b.nb = (int)ipow(p->rad[1], p->m - 1);
    b.rows = p->b_rows;
    b.d0max = p->dmax[0];
    b.emax = p->b_emax;
    b.ew = p->b_ew;
    b.sw = p->b_sw;
    b.gamma = p->d.gamma;
    b.cvar0 = p->d.c_var[0];
    b.cvar1 = p->d.c_var[1];
    b.z = p->dev.z;
    b.pmf0 = p->dev.pmf;
    b.rexp0 = p->dev.rexp0;
    b.e_pmf = p->dev.epmf;
    b.e_cdf = p->dev.ecdf;
    b.e_tail = p->dev.etail;
    b.rexp1 = p->dev.rexp1;
    b.tiled = p->b_tiled ? 1 : 0;
    b.nw = (int)ipow(p->rad[0], p->m - 2);
    b.ewp = p->b_ewp;
    b.ppad = p->dev.bppad;
    b.gpad = p->dev.bgpad;
    b.ctl = p->dev.ctl;
    b.partials = p->dev.partials;
    b.pi = p->dev.pi;
    b.gap = p->dev.gap;
    return b;
}

static B1Dev make_b1dev(const pvi_mdp* p) {
    B1Dev b{};
    const int m = p->m;
    b.m = m;
    b.Ra = p->rad[0];
    b.Rb = p->rad[1];
    b.HA = p->b1_ha;
    b.HB = p->b1_hb;
    b.na1 = (int)ipow(b.Ra, m - 1);
    b.nb1 = (int)ipow(b.Rb, m - 1);
    b.NA = (int)ipow(b.Ra, m);
    b.NB = (int)ipow(b.Rb, m);
    b.gw = std::max(1, std::min(b.na1, 4096 / std::max(1, b.nb1)));
    // the final stage keeps cb orders' W slices (rows of cbp doubles) and three demand
    // tables in 64 KB of LDS
    auto stride = [](int cb) {
        int c = (cb + 1) / 2 * 2;
        return c % 4 == 0 ? c + 2 : c;
    };
    b.cb = std::min(16, b.Rb);
    while (b.cb > 1 && (int64_t)b.na1 * stride(b.cb) + 3 * (b.HA + 1) > 8192) --b.cb;
    b.cbp = stride(b.cb);
    // PVI_B1_LANES=0 keeps the final kernel over lanes of x_a for every sweep (for tests:
    // both give the same values)
    const char* lanes = std::getenv("PVI_B1_LANES");
    b.lanes_ab = lanes && std::strcmp(lanes, "0") == 0 ? 0 : 1;
    b.gamma = p->d.gamma;
    b.cva = p->d.c_var[0];
    b.cvb = p->d.c_var[1];
    const auto& d = p->dev;
    b.w = d.b1w;
    b.y = d.b1y;
    b.pa1 = d.b1pa;
    b.fa = d.b1fa;
    b.ga = d.b1ga;
    b.pb = d.b1pb;
    b.fb = d.b1fb;
    b.j = d.b1j;
    b.jc = d.b1jc;
    b.rev = d.b1rev;
    b.xb_order = d.b1xb;
    b.ctl = d.ctl;
    b.partials = d.partials;
    b.nslots = family_tiles(p);
    b.pi = d.pi;
    b.gap = d.gap;
    return b;
}

hipError_t family_initial_values(pvi_mdp* p, double* v, hipStream_t s) {
    if (p->family != PVI_FAMILY_SUBST2_L1) return hipErrorInvalidValue;
    return launch_b1_initial(make_b1dev(p), v, s);
}

static CDev make_cdev(const pvi_mdp* p) {
    CDev c{};
    const int R = p->rad[0];
    c.R = R;
    c.m = p->m;
    c.P = p->P;
    c.nzu = (int)ipow(R, p->m - 2);
    c.nblk = ipow(R, p->m - 1);
    c.npair = p->c_npair;
    c.tab = p->c_tab;
    c.xt = p->c_xt;
    c.lpmax = p->c_lpmax;
    c.dmax = p->dmax[0];
    for (int i = 0; i < 10; ++i) c.pow_r[i] = (int)ipow(R, i);
    c.gamma = p->d.gamma;
    c.cfixed = p->d.c_fixed;
    const auto& d = p->dev;
    c.u = d.cu;
    c.t0 = d.ct0;
    c.t1 = d.ct1;
    c.tf = d.ctf;
    std::memcpy(c.lb, p->c_lb, sizeof(c.lb));
    c.exogenous = p->c_exogenous ? 1 : 0;
    c.alim = R - 1;
    c.top_only = 0;
    c.pmf = d.cpmf;
    c.cdf = d.ccdf;
    c.tail = d.ctail;
    c.r0 = d.cr0;
    c.binq = d.cbinq;
    c.binm = d.cbinm;
    c.pair_y = d.cpy;
    c.pair_r = d.cpr;
    c.pair_base = d.cpb;
    c.ctl = d.ctl;
    c.partials = d.partials;
    c.pi = d.pi;
    c.gap = d.gap;
    return c;
}

static size_t c_table_entries(const pvi_mdp* p) {  // entries of one merge table
    return (size_t)p->P * p->c_npair * ipow(p->rad[0], p->m - 1);
}

std::string family_support_msg(const pvi_mdp* p) {
    if (p->family == PVI_FAMILY_LEADTIME) return "ok";
    if (p->family == PVI_FAMILY_SUBST2) {
        if (p->m < 2) return "scenario B needs m >= 2 on the GPU";
        if (p->rad[1] > PVI_B_R1MAX) return "scenario B needs a_max[1] <= 15 on the GPU";
        const size_t lds = sizeof(double) * ((size_t)p->b_rows * (PVI_B_R1MAX + 2) + p->dmax[0] + 65);
        if (lds > 65536) return "scenario B stage-2 table exceeds LDS (too many product-0 states)";
        return "ok";
    }
    if (p->family == PVI_FAMILY_RUL_WEEKDAY) {
        if (p->ns > (int64_t(1) << 31))
            return "more than 2^31 states: this scenario-C handle serves heuristic rollouts only";
        if (p->m > 9) return "scenario C needs m <= 9 on the GPU";
        const size_t lds = sizeof(double) * ((size_t)p->c_lpmax + 3 * (size_t)p->c_tab);
        if (lds > 65536) return "scenario C demand table exceeds LDS";
        return "ok";
    }
    if (p->family == PVI_FAMILY_SUBST2_L1) {
        const int64_t na1 = ipow(p->rad[0], p->m - 1), nb1 = ipow(p->rad[1], p->m - 1);
        if (ipow(p->rad[1], p->m) > 65535)
            return "the lead-time-1 two-product family needs (a_max[1]+1)^m <= 65535 on the GPU";
        if (2 * na1 + 3 * (p->b1_ha + 1) > 8192 || nb1 > 4096)
            return "the lead-time-1 two-product family: aged stock of one product exceeds LDS";
        return "ok";
    }
    return "this family has no GPU kernel yet";
}

bool family_supported(const pvi_mdp* p) { return family_support_msg(p) == "ok"; }

int family_tiles(const pvi_mdp* p) {
    if (p->family == PVI_FAMILY_LEADTIME) {
        const int R = p->rad[0];
        if (p->d.issuing == PVI_LIFO && p->m >= 2)  // one partial per LIFO tile
            return (int)(ipow(R, p->L - 1) * ipow(R, p->m - 2));
        return p->a_G > 0 ? (int)(p->a_groups.size() / p->a_G) : 1;  // one per tile group
    }
    if (p->family == PVI_FAMILY_SUBST2)  // one per (product-1 stock, middle product-0 digits)
        return (int)(ipow(p->rad[1], p->m - 1) * (p->b_tiled ? ipow(p->rad[0], p->m - 2) : 1));
    if (p->family == PVI_FAMILY_RUL_WEEKDAY) {
        if (p->m >= 4 && p->c_exogenous)  // top merge fused with the final sum
            return (int)c_partial_slots(p->P, ipow(p->rad[0], p->m - 2));
        return (int)(p->P * ((ipow(p->rad[0], p->m - 1) + 255) / 256));
    }
    if (p->family == PVI_FAMILY_SUBST2_L1)  // either final kernel's grid fits
        return (int)(ipow(p->rad[1], p->m) *
                     std::max((ipow(p->rad[0], p->m) + 255) / 256,
                              (ipow(p->rad[0], p->m - 1) + kB1Groups - 1) / kB1Groups));
    return 1;
}

static size_t b1_w_entries(const pvi_mdp* p) {
    return (size_t)p->na * ipow(p->rad[1], p->m) * ipow(p->rad[0], p->m - 1);
}

static size_t b1_y_entries(const pvi_mdp* p) {
    return (size_t)p->na * p->b1_hb * ipow(p->rad[0], p->m);
}

size_t family_extra_bytes(const pvi_mdp* p) {
    if (p->family == PVI_FAMILY_LEADTIME)
        return sizeof(double) * (3 * (size_t)p->tab + p->a_r0.size()) +
               sizeof(int32_t) * p->a_groups.size();
    if (p->family == PVI_FAMILY_SUBST2)
        return sizeof(double) * ((size_t)p->b_rows * ipow(p->rad[1], p->m) + p->b_rexp0.size() +
                                 3 * p->b_epmf.size() + p->b_rexp1.size() + p->pmf[0].size() +
                                 p->b_ppad.size() + p->b_gpad.size());
    if (p->family == PVI_FAMILY_RUL_WEEKDAY) {
        const size_t ut = (size_t)p->ns * p->rad[0];
        const size_t tt = p->m >= 3 ? c_table_entries(p) : 0;
        const size_t ntab = p->c_exogenous ? 2 : 3;
        return sizeof(double) * (ut + ntab * tt + 3 * p->c_pmf.size() + p->c_r0.size() +
                                 p->c_binq.size() + p->c_binm.size());
    }
    if (p->family == PVI_FAMILY_SUBST2_L1)
        return sizeof(double) * (b1_w_entries(p) + b1_y_entries(p) + 3 * p->b1_pa1.size() +
                                 p->b1_pb.size() + p->b1_fb.size() +
                                 p->b1_j.size() + p->b1_jc.size() + p->b1_rev.size());
    return 0;
}

// The stock vectors x_b of product b ordered by their digit sum I_b (stable): the final
// kernels take x_b in this order, so the workgroups that read one I_b slice of the Y
// table (Ra Rb NA values) run together and find it in the caches.
static std::vector<int32_t> b1_xb_order(const pvi_mdp* p) {
    const int R = p->rad[1], m = p->m;
    const int64_t nb = ipow(R, m);
    std::vector<int32_t> order((size_t)nb);
    std::vector<int> sum((size_t)nb);
    for (int64_t x = 0; x < nb; ++x) {
        int t = 0;
        for (int64_t v = x, k = 0; k < m; ++k, v /= R) t += (int)(v % R);
        sum[(size_t)x] = t;
        order[(size_t)x] = (int32_t)x;
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return sum[(size_t)a] < sum[(size_t)b]; });
    return order;
}

// A demand table of product a followed by kB1Pad zeros: the final kernel over lanes of b's
// orders reads it at x_1 + k for every x_1 < 16, also past a's largest issue.
static std::vector<double> padded(const std::vector<double>& v) {
    std::vector<double> out(v);
    out.resize(v.size() + kB1Pad, 0.0);
    return out;
}

template <class T>
static hipError_t upload_vec(T** dst, const std::vector<T>& src) {
    hipError_t e = hipMalloc((void**)dst, sizeof(T) * std::max<size_t>(src.size(), 1));
    if (e != hipSuccess || src.empty()) return e;
    return hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
}

// Merge block widths chosen by timing, per (R, m, number of weekdays), shared by every
// handle of the process.  PVI_TUNE=0 in the environment keeps the LDS rule instead.
namespace {
using TuneKey = std::tuple<int, int, int>;
using TuneVal = std::array<std::array<int32_t, 10>, 2>;
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;

pvi_status tune_c(pvi_mdp* p) {
    std::memset(p->c_lb, 0, sizeof(p->c_lb));
    // PVI_C_BLOCK=<width>: that block width at every merge level where it fits
    const char* force = std::getenv("PVI_C_BLOCK");
    if (force) {
        const int w = std::atoi(force);
        if (w != 4 && w != 8 && w != 12 && w != 16 && w != 32)
            return fail(PVI_E_INVALID, "PVI_C_BLOCK must be 4, 8, 12, 16 or 32");
        const int R = p->rad[0], rc = R <= 8 ? 8 : R <= 16 ? 16 : R <= 24 ? 24 : 32;
        for (int a = 0; a < 2; ++a) {
            for (int j = 3; j < 10; ++j) {
                const bool fused = j == p->m - 1 && p->c_exogenous;
                const bool fits = (size_t)(a ? 4 : 8) * R * rc * w <= 65536 &&
                                  R * w <= (fused ? kCFusedThreads : 1024);
                p->c_lb[a][j] = fits ? w : 0;
            }
        }
        return PVI_OK;
    }
    const char* env = std::getenv("PVI_TUNE");
    if ((env && std::strcmp(env, "0") == 0) || p->m < 4) return PVI_OK;
    const TuneKey key{p->rad[0], p->m, p->P};
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune.find(key);
    if (it == g_tune.end()) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
            return fail(PVI_E_DEVICE, "scenario C tuning: stream creation failed");
        int32_t lb[2][10];
        const hipError_t e = tune_c_merge(make_cdev(p), s, lb);
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
        if (e != hipSuccess)
            return fail(PVI_E_DEVICE, std::string("scenario C tuning: ") + hipGetErrorString(e));
        TuneVal v{};
        for (int a = 0; a < 2; ++a)
            for (int j = 0; j < 10; ++j) v[a][j] = lb[a][j];
        it = g_tune.emplace(key, v).first;
        const char* verbose = std::getenv("PVI_TUNE_VERBOSE");
        if (verbose && std::strcmp(verbose, "1") == 0) {
            std::fprintf(stderr, "pvi: scenario C R=%d m=%d P=%d merge block widths", p->rad[0],
                         p->m, p->P);
            for (int j = 3; j <= p->m - 1 && j < 10; ++j)
                std::fprintf(stderr, " j=%d: fp64 %d fp32 %d;", j, lb[0][j], lb[1][j]);
            std::fprintf(stderr, "\n");
        }
    }
    for (int a = 0; a < 2; ++a)
        for (int j = 0; j < 10; ++j) p->c_lb[a][j] = it->second[a][j];
    return PVI_OK;
}
}  // namespace

// Tiles per wavefront (G) and path points per staged chunk (CH) of the scenario-A
// FIFO backup, chosen by timing at the first solve of a shape (R, m, L) in a process
// and kept for every later handle of that shape.  Candidates: G = floor(64 / R), 2
// and 1, each with the longest chunk its staging lanes allow and half of it; each is
// timed over three FP64 sweeps (after one untimed) on this handle's buffers, with
// the stopping rule off.  PVI_TUNE=0 keeps the rule of build_a_work_list;
// PVI_A_GROUP and PVI_A_CHUNK fix the choice.  Results do not depend on it.
namespace {
std::mutex g_tune_a_mu;
std::map<TuneKey, std::pair<int, int>> g_tune_a;

pvi_status tune_a(pvi_mdp* p) {
    const char* env = std::getenv("PVI_TUNE");
    if ((env && std::strcmp(env, "0") == 0) || std::getenv("PVI_A_GROUP") ||
        std::getenv("PVI_A_CHUNK") || (p->d.issuing == PVI_LIFO && p->m >= 2))
        return PVI_OK;
    const TuneKey key{p->rad[0], p->m, p->L};
    std::lock_guard<std::mutex> lock(g_tune_a_mu);
    auto it = g_tune_a.find(key);
    if (it == g_tune_a.end()) {
        auto& d = p->dev;
        std::vector<std::pair<int, int>> cand;
        const int gmax = a_group_max(p);
        for (int G : {gmax, std::min(gmax, 2), 1})
            for (int CH : {a_chunk_max(p, G), std::max(1, a_chunk_max(p, G) / 2)})
                if (std::find(cand.begin(), cand.end(), std::make_pair(G, CH)) == cand.end())
                    cand.emplace_back(G, CH);
        hipStream_t s = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        int32_t* groups = nullptr;
        double* parts = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e == hipSuccess) e = launch_fill(d.v64[0], 0.0, p->ns, s);
        // one fixed-length sweep after another: the stop flag is never set
        Ctl zero{};
        if (e == hipSuccess) e = hipMemcpyAsync(d.ctl, &zero, sizeof(Ctl), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        float best = 1e30f;
        std::pair<int, int> choice{p->a_G, p->a_CH};
        for (const auto& c : cand) {
            if (e != hipSuccess) break;
            build_a_work_list(p, c.first, c.second);
            const int ng = (int)(p->a_groups.size() / p->a_G);
            if (groups) (void)hipFree(groups);
            if (parts) (void)hipFree(parts);
            groups = nullptr;
            parts = nullptr;
            if ((e = upload_vec(&groups, p->a_groups)) != hipSuccess ||
                (e = hipMalloc((void**)&parts, sizeof(double) * 4 * (size_t)ng)) != hipSuccess)
                break;
            ADev a = make_adev(p);
            a.groups = groups;
            a.partials = parts;
            a.v_in = d.v64[0];
            a.v_out = d.v64[1];
            a.fixed = 1;
            if ((e = launch_backup_a(a, 0, 0, 0, s)) != hipSuccess ||
                (e = hipEventRecord(e0, s)) != hipSuccess)
                break;
            for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch_backup_a(a, 0, 0, 0, s);
            if (e != hipSuccess || (e = hipEventRecord(e1, s)) != hipSuccess ||
                (e = hipEventSynchronize(e1)) != hipSuccess)
                break;
            float ms = 0.f;
            if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
            if (ms < best) {
                best = ms;
                choice = c;
            }
        }
        if (groups) (void)hipFree(groups);
        if (parts) (void)hipFree(parts);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s) (void)hipStreamDestroy(s);
        if (e != hipSuccess)
            return fail(PVI_E_DEVICE, std::string("scenario A tuning: ") + hipGetErrorString(e));
        it = g_tune_a.emplace(key, choice).first;
        const char* verbose = std::getenv("PVI_TUNE_VERBOSE");
        if (verbose && std::strcmp(verbose, "1") == 0)
            std::fprintf(stderr, "pvi: scenario A R=%d m=%d L=%d: G=%d CH=%d (%.1f us per sweep)\n",
                         p->rad[0], p->m, p->L, choice.first, choice.second, 1e3f * best / 3.f);
    }
    if (p->a_G != it->second.first || p->a_CH != it->second.second)
        build_a_work_list(p, it->second.first, it->second.second);
    return PVI_OK;
}
}  // namespace

pvi_status family_init(pvi_mdp* p) {
    auto& d = p->dev;
    if (p->family == PVI_FAMILY_LEADTIME) {
        pvi_status st = tune_a(p);
        if (st != PVI_OK) return st;
        // the chosen work list may have more groups than the partials were sized for
        const int nt = family_tiles(p);
        if (nt > d.tiles) {
            (void)hipFree(d.partials);
            d.partials = nullptr;
            if (hipMalloc((void**)&d.partials, 4 * sizeof(double) * (size_t)nt) != hipSuccess)
                return fail(PVI_E_NOMEM, "scenario A partials allocation failed");
        }
        d.tiles = nt;
        if (upload_vec(&d.agroups, p->a_groups) != hipSuccess)
            return fail(PVI_E_NOMEM, "scenario A work list allocation failed");
    }
    if (p->family == PVI_FAMILY_SUBST2) {
        const size_t zn = (size_t)p->b_rows * ipow(p->rad[1], p->m);
        if (hipMalloc((void**)&d.z, sizeof(double) * zn) != hipSuccess ||
            upload_vec(&d.pmf, p->pmf[0]) != hipSuccess ||
            upload_vec(&d.rexp0, p->b_rexp0) != hipSuccess ||
            upload_vec(&d.epmf, p->b_epmf) != hipSuccess ||
            upload_vec(&d.ecdf, p->b_ecdf) != hipSuccess ||
            upload_vec(&d.etail, p->b_etail) != hipSuccess ||
            upload_vec(&d.rexp1, p->b_rexp1) != hipSuccess ||
            (p->b_tiled && (upload_vec(&d.bppad, p->b_ppad) != hipSuccess ||
                            upload_vec(&d.bgpad, p->b_gpad) != hipSuccess)))
            return fail(PVI_E_NOMEM, "scenario B table allocation failed");
    }
    if (p->family == PVI_FAMILY_RUL_WEEKDAY) {
        const size_t ut = (size_t)p->ns * p->rad[0];
        const size_t tt = p->m >= 3 ? c_table_entries(p) : 1;
        if (hipMalloc(&d.cu, sizeof(double) * ut) != hipSuccess ||
            hipMalloc(&d.ct0, sizeof(double) * tt) != hipSuccess ||
            hipMalloc(&d.ct1, sizeof(double) * tt) != hipSuccess ||
            (!p->c_exogenous && hipMalloc(&d.ctf, sizeof(double) * tt) != hipSuccess) ||
            upload_vec(&d.cpmf, p->c_pmf) != hipSuccess ||
            upload_vec(&d.ccdf, p->c_cdf) != hipSuccess ||
            upload_vec(&d.ctail, p->c_tail) != hipSuccess ||
            upload_vec(&d.cr0, p->c_r0) != hipSuccess ||
            upload_vec(&d.cbinq, p->c_binq) != hipSuccess ||
            upload_vec(&d.cbinm, p->c_binm) != hipSuccess ||
            upload_vec(&d.cpy, p->c_pair_y) != hipSuccess ||
            upload_vec(&d.cpr, p->c_pair_r) != hipSuccess ||
            upload_vec(&d.cpb, p->c_pair_base) != hipSuccess)
            return fail(PVI_E_NOMEM, "scenario C table allocation failed");
        const pvi_status st = tune_c(p);
        if (st != PVI_OK) return st;
    }
    if (p->family == PVI_FAMILY_SUBST2_L1) {
        if (hipMalloc((void**)&d.b1w, sizeof(double) * b1_w_entries(p)) != hipSuccess ||
            hipMalloc((void**)&d.b1y, sizeof(double) * b1_y_entries(p)) != hipSuccess ||
            upload_vec(&d.b1pa, padded(p->b1_pa1)) != hipSuccess ||
            upload_vec(&d.b1fa, padded(p->b1_fa)) != hipSuccess ||
            upload_vec(&d.b1ga, padded(p->b1_ga)) != hipSuccess ||
            upload_vec(&d.b1pb, p->b1_pb) != hipSuccess ||
            upload_vec(&d.b1fb, p->b1_fb) != hipSuccess ||
            upload_vec(&d.b1j, p->b1_j) != hipSuccess ||
            upload_vec(&d.b1jc, p->b1_jc) != hipSuccess ||
            upload_vec(&d.b1rev, p->b1_rev) != hipSuccess ||
            upload_vec(&d.b1xb, b1_xb_order(p)) != hipSuccess)
            return fail(PVI_E_NOMEM, "lead-time-1 two-product table allocation failed");
    }
    return PVI_OK;
}

void family_free(pvi_mdp* p) {
    auto& d = p->dev;
    void* bufs[] = {d.z,    d.rexp0, d.epmf,  d.ecdf,  d.etail, d.rexp1, d.cu,  d.ct0,
                    d.ct1,  d.cpmf,  d.ccdf,  d.ctail, d.cr0,   d.cbinq,  d.cbinm, d.cpy,
                    d.cpr,  d.cpb, d.agroups, d.ctf, d.b1w, d.b1y, d.b1pa, d.b1fa, d.b1ga,
                    d.b1pb, d.b1fb, d.b1j, d.b1jc, d.b1rev, d.b1xb, d.bppad, d.bgpad};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    d.b1w = d.b1y = d.b1pa = d.b1fa = d.b1ga = d.b1pb = d.b1fb = d.b1j = d.b1jc = d.b1rev =
        nullptr;
    d.b1xb = nullptr;
    d.z = d.rexp0 = d.epmf = d.ecdf = d.etail = d.rexp1 = d.bppad = d.bgpad = nullptr;
    d.cu = d.ct0 = d.ct1 = d.ctf = nullptr;
    d.cpmf = d.ccdf = d.ctail = d.cr0 = d.cbinq = d.cbinm = nullptr;
    d.cpy = d.cpr = d.cpb = nullptr;
    d.agroups = nullptr;
}

// No family fuses the span today: a device-wide release fence per workgroup (needed
// for a last-workgroup reduction) writes back L2 on every XCD and cost more than
// the separate single-workgroup span launch it would save.
bool family_fused_span(const pvi_mdp*) { return false; }

static hipError_t family_backup_launch(pvi_mdp* p, int fp32, int kahan, int extract, int fixed,
                                       const void* vin, void* vout, hipStream_t s);

hipError_t family_backup(pvi_mdp* p, int fp32, int kahan, int extract, int fixed,
                         const void* vin, void* vout, hipStream_t s, hipEvent_t ev0,
                         hipEvent_t ev1) {
    if (p->family == PVI_FAMILY_LEADTIME) {
        ADev a = make_adev(p);
        if (!a.lifo) {
            // the FIFO kernel takes the events with its launch (no separate stream packets)
            a.v_in = vin;
            a.v_out = vout;
            a.fixed = fixed;
            return launch_backup_a(a, fp32, kahan, extract, s, ev0, ev1);
        }
    }
    hipError_t e;
    if (ev0 && (e = hipEventRecord(ev0, s)) != hipSuccess) return e;
    if ((e = family_backup_launch(p, fp32, kahan, extract, fixed, vin, vout, s)) != hipSuccess)
        return e;
    return ev1 ? hipEventRecord(ev1, s) : hipSuccess;
}

// The backup of every family other than scenario-A FIFO (that one too, without events).
static hipError_t family_backup_launch(pvi_mdp* p, int fp32, int kahan, int extract, int fixed,
                                       const void* vin, void* vout, hipStream_t s) {
    if (p->family == PVI_FAMILY_LEADTIME) {
        ADev a = make_adev(p);
        a.v_in = vin;
        a.v_out = vout;
        a.fixed = fixed;
        if (a.lifo) return launch_backup_a_lifo(a, fp32, extract, s);
        return launch_backup_a(a, fp32, kahan, extract, s, nullptr, nullptr);
    }
    if (p->family == PVI_FAMILY_SUBST2) {
        BDev b = make_bdev(p);
        b.v_in = vin;
        b.v_out = vout;
        b.extract = extract;
        return launch_backup_b(b, fp32, extract, s);
    }
    if (p->family == PVI_FAMILY_RUL_WEEKDAY) {
        CDev c = make_cdev(p);
        c.v_in = vin;
        c.v_out = vout;
        c.extract = extract;
        return launch_backup_c(c, fp32, extract, s);
    }
    if (p->family == PVI_FAMILY_SUBST2_L1) {
        B1Dev b = make_b1dev(p);
        b.v_in = vin;
        b.v_out = vout;
        b.extract = extract;
        return launch_backup_b1(b, fp32, extract, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace pvi
