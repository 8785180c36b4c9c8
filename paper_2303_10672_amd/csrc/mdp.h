// The pvi_mdp handle: validated descriptor, host tables, device buffers, results.
#pragma once

#include <hip/hip_runtime_api.h>

#include <atomic>
#include <cstdint>
#include <mutex>
#include <vector>

#include "pvi_internal.h"

struct pvi_mdp {
    pvi_mdp_desc d{};    // copy of the descriptor (table pointers cleared)
    int family = 0, m = 0, L = 0, P = 1;
    int rad[2] = {1, 1};   // radix per product (a_max + 1)
    int dmax[2] = {0, 0};
    int ndig = 0;
    int radix[16] = {0};
    int64_t ns = 0;
    int na = 0;
    std::vector<double> pmf[2];  // [P][dmax+1] FP64 demand PMF per product
    std::vector<double> life;    // C: [(a_max+1) * m], p_k(a) at a*m + k-1

    // Scenario A kernel tables
    int tab = 0, xt = 0;
    std::vector<double> a_pmf, a_cdf, a_tail, a_r0;
    // scenario-A kernel work list: groups of a_G tiles with one digit sum each
    // (-1 pads a short group), a_CH path points staged per chunk
    std::vector<int32_t> a_groups;
    int a_G = 0, a_CH = 0;

    // Scenario B kernel tables
    int b_rows = 0, b_emax = 0, b_ew = 0, b_sw = 0;
    std::vector<double> b_rexp0, b_epmf, b_ecdf, b_etail, b_rexp1;
    // tiled sweep kernels (shape within their compile-time bounds): rows of the
    // product-1 demand PMF and tail, zero-padded to b_ewp entries
    bool b_tiled = false;
    int b_ewp = 0;
    std::vector<double> b_ppad, b_gpad;

    // Scenario C kernel tables
    bool c_exogenous = true;
    int32_t c_lb[2][10] = {};  // merge block width per [FP32 storage][level] (0: LDS rule)
    int c_tab = 0, c_xt = 0, c_lpmax = 0, c_npair = 0;
    std::vector<double> c_pmf, c_cdf, c_tail, c_r0, c_binq, c_binm;
    std::vector<int32_t> c_pair_y, c_pair_r, c_pair_base;

    // Scenario B as the paper runs it (lead time 1): issue probabilities and revenue
    int b1_ha = 0, b1_hb = 0;  // m a_max + 1 per product
    std::vector<double> b1_pa, b1_pb, b1_fb, b1_j, b1_jc, b1_rev;
    std::vector<double> b1_pa1, b1_fa, b1_ga;  // [HA + 1] P(D_a = h), P(D_a <= h), P(D_a >= h)

    int64_t logical_per_sweep = 0;
    int64_t executed_per_sweep = 0;

    // device state (allocated on the first solve)
    struct Dev {
        bool ready = false;
        int device = -1;
        hipStream_t own = nullptr;
        double* v64[2] = {nullptr, nullptr};
        // extra FP64 value tables of the periodic rule's ring (slots 2 .. period),
        // taken at the first solve that needs them
        double* vring[8] = {};
        double* pparts = nullptr;  // periodic test partials
        float* v32[2] = {nullptr, nullptr};
        int32_t* pi = nullptr;
        double* gap = nullptr;
        double* partials = nullptr;
        pvi::Ctl* ctl = nullptr;
        pvi::Ctl* h_ctl = nullptr;  // pinned host mirror
        double *pmf = nullptr, *cdf = nullptr, *tail = nullptr, *r0 = nullptr;
        int32_t* agroups = nullptr;
        double *z = nullptr, *rexp0 = nullptr, *epmf = nullptr, *ecdf = nullptr,
               *etail = nullptr, *rexp1 = nullptr, *bppad = nullptr, *bgpad = nullptr;
        void *cu = nullptr, *ct0 = nullptr, *ct1 = nullptr, *ctf = nullptr;
        double *cpmf = nullptr, *ccdf = nullptr, *ctail = nullptr, *cr0 = nullptr,
               *cbinq = nullptr, *cbinm = nullptr;
        int32_t *cpy = nullptr, *cpr = nullptr, *cpb = nullptr;
        double *b1w = nullptr, *b1y = nullptr, *b1pa = nullptr, *b1fa = nullptr, *b1ga = nullptr,
               *b1pb = nullptr, *b1fb = nullptr, *b1j = nullptr, *b1jc = nullptr,
               *b1rev = nullptr;
        int32_t* b1xb = nullptr;  // x_b in the final kernels' order (by digit sum I_b)
        int tiles = 0;
        size_t bytes = 0;
        std::vector<hipEvent_t> ev;
        hipEvent_t span_ev[2] = {nullptr, nullptr};  // a whole solve's stream time
        // instantiated graphs of kGraphSweeps sweeps (backup + span launches), keyed by
        // storage precision, compensated sums and fixed-length runs; their kernel
        // arguments hold this handle's buffers, so they live and die with them
        struct SweepGraph {
            int key = -1;
            hipGraphExec_t exec = nullptr;
        };
        std::vector<SweepGraph> graphs;
    } dev;

    // results of the last solve; have_result = 2 means they are in the host
    // vectors below (batched solves of the request server)
    std::vector<double> h_v, h_gap;
    std::vector<int32_t> h_pi;
    int have_result = 0;
    int ret_buf = 0;  // value-table slot holding V (0, 1: v64; 2..: dev.vring)
    std::mutex mu;
};

namespace pvi {
pvi_status ensure_device(pvi_mdp* p);
void free_device(pvi_mdp* p);
pvi_status park_results(pvi_mdp* p);
// vi_solve with a switch for the captured sweep graphs (off: every sweep launched
// directly) and an optional progress counter (sweeps completed, stored at every
// host check)
pvi_status solve_impl(pvi_mdp* p, const pvi_solve_opts* opts, pvi_result* res, bool graphs,
                      std::atomic<int>* progress);
size_t device_bytes(const pvi_mdp* p);
// Scenario-A work list for G tiles per wavefront and CH path points per staged chunk
// (0: the default rule); the largest G and CH the kernel takes.
void build_a_work_list(pvi_mdp* p, int G, int CH);
int a_group_max(const pvi_mdp* p);
int a_chunk_max(const pvi_mdp* p, int G);
pvi::ADev make_adev(const pvi_mdp* p);
// Shift from V to the midpoint of MacQueen's bounds on V* (the standard bounds of
// discounted value iteration, V + gamma/(1-gamma) [dmin, dmax] with dmax, dmin the last
// sweep's largest and smallest increment): gamma/(1-gamma) times the increments' mean;
// 0 for gamma = 1, where the bounds do not apply.
inline double vhat_shift(double gamma, double dmax, double dmin) {
    return gamma < 1.0 ? gamma / (1.0 - gamma) * 0.5 * (dmax + dmin) : 0.0;
}
}  // namespace pvi
