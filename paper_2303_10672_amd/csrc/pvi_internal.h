// Internal definitions shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "pvi.h"

namespace pvi {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
pvi_status fail(pvi_status st, const std::string& msg);

#define PVI_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            return ::pvi::fail(PVI_E_DEVICE, std::string(#call) + ": " +           \
                                                 hipGetErrorString(e_));           \
    } while (0)

// ------------------------------------------------------------------ device control
// One per solve, in device memory.  Written only by the single-workgroup span
// kernel and by the host between launches; read by every backup launch.
struct Ctl {
    double mu;        // FP32 storage: centre shift applied to the next sweep
    double c;         // FP32 storage: FP64 offset of the current iterate, V = c + v
    double dmax, dmin;  // max/min of V_new - V of the last sweep
    double span;      // dmax - dmin
    double best_span; // smallest span seen in the current phase
    double thr;       // stopping threshold on the span (negative: never stop)
    double floor32;   // FP32 phase ends when span <= max(thr, floor32 * max|v|)
    double vabs;      // FP32 storage: max |v| of the last sweep
    int32_t stop;     // 1 once the phase's stopping rule fired; later launches return
    int32_t sweeps;   // sweeps completed in the current phase
    int32_t stop_sweep;
    int32_t stall;    // sweeps without a new best span (FP32 phase)
    int32_t fp32_phase;
    int32_t rule;     // 0: span rule, 1: sup-norm rule max|V_new - V| < thr,
                      // 2: periodic rule (decided by the periodic check kernels)
    int32_t pad[2];
};

// ------------------------------------------------------------------ family A
struct ADev {
    const void* v_in;
    void* v_out;
    int32_t* pi;        // extraction only
    double* gap;        // extraction only
    double* partials;   // [ngroups][4]: max dv, min dv, max v_out, min v_out
    const double* r0;   // [R][xt]: expected one-day reward without the order cost
    const double* pmf;  // [tab]: P(d), zero beyond d_max
    const double* cdf;  // [tab]: P(D <= d), one beyond d_max
    const double* tail; // [tab]: P(D >= d), zero beyond d_max
    Ctl* ctl;
    int64_t stride_a;   // R^(m+L-2): offset of next-state block of action a
    int64_t stride_h;   // R^(m-1): block size, one block per in-transit vector
    int32_t R, m, dmax, xt, tab;
    int32_t nz;         // R^(m-2) tiles per in-transit vector (1 if m <= 2)
    int32_t r2;         // R if m >= 2 else 1
    int32_t tiles;      // nh * nz
    const int32_t* groups;  // [ngroups][G] tile ids, equal digit sum per group, -1 = none
    int32_t G, CH, ngroups; // tiles per wavefront, path points per staged chunk
    int32_t pow_y[8];   // R^(i-1), weight of next-state digit i inside a block
    int32_t fixed;      // 1: fixed number of sweeps, the stopping rule is not applied
    int32_t lifo;       // 1: LIFO issuing (tiles are (O, X_{m-1}..X_2) then)
    int32_t lmax;       // LIFO: longest backwards depletion list, (m-2)(R-1) + R
    double gamma, cvar;
};

// ------------------------------------------------------------------ family B
#define PVI_B_R1MAX 16  // product-1 order choices per kernel row (a_max[1] <= 15)
#define PVI_B_JMAX 32   // tiled scenario-B kernels: product-0 demand values (d_max[0] <= 31)
struct BDev {
    const void* v_in;
    void* v_out;
    int32_t* pi;
    double* gap;
    double* partials;   // [nb][4]
    double* z;          // [rows][nb * r1] stage-1 table
    const double* pmf0;   // [d0max+1]
    const double* rexp0;  // [stock0]: c_rev0 E[min(d0, stock0)]
    const double* e_pmf;  // [d0max+1][ew]: product-1 demand incl. substitutes, given u0
    const double* e_cdf;
    const double* e_tail;
    const double* rexp1;  // [d0max+1][sw]: c_rev1 E[min(e, stock1) | u0]
    const double* ppad;   // [d0max+1][ewp]: e_pmf rows, zero past emax (tiled kernels)
    const double* gpad;   // [d0max+1][ewp]: e_tail rows, zero past emax
    Ctl* ctl;
    int32_t m, r0, r1, r1pad, na, nb, rows, d0max, emax, ew, sw, extract;
    int32_t tiled;  // sweeps use the tiled kernels (one partial per (ib, middle digits))
    int32_t nw;     // r0^(m-2): middle product-0 digit combinations
    int32_t ewp;
    double gamma, cvar0, cvar1;
};


// ------------------------------------------------------------------ family C
struct CDev {
    const void* v_in;
    void* v_out;
    int32_t* pi;
    double* gap;
    double* partials;     // [P * ceil(nblk/256)][4]
    void* u;              // U[tau][z_m][z_{m-1}..z_1]
    void* t0;             // merge ping-pong tables [tau][(y_m, r)][digits]
    void* t1;
    void* tf;             // order-dependent life: top-level rows r = a - y_m of every a
    const double* pmf;    // [P][tab] per-weekday demand, zero past d_max
    const double* cdf;    // [P][tab], one past d_max
    const double* tail;   // [P][tab], zero past d_max
    const double* r0;     // [P][R][xt] expected one-day reward of post-arrival stock
    const double* binq;   // [m][R][R] Bin(y; r, q_j) (for one order size a when the
                          // life distribution depends on it)
    const double* binm;   // [R][R] Bin(y; a, p_m(a))
    const int32_t* pair_y;
    const int32_t* pair_r;
    const int32_t* pair_base;
    Ctl* ctl;
    int64_t nblk;         // R^(m-1) states per weekday
    int32_t R, m, P, nzu, npair, tab, xt, lpmax, dmax, extract;
    int32_t lb[2][10];    // merge block width per [FP32 storage][level j] (0: the LDS rule)
    int32_t exogenous;    // 0: one merge chain per order size a
    int32_t alim;         // merges compute rows with y_m + r <= alim
    int32_t top_only;     // and, when set, only the row r = alim - y_m
    int32_t pow_r[10];
    double gamma, cfixed;
};

// ------------------------------------------------------------------ family B, lead time 1
struct B1Dev {
    const void* v_in;
    void* v_out;
    int32_t* pi;
    double* gap;
    double* partials;     // [nslots][4]
    int32_t nslots;       // NB * max(ceil(NA / 256), ceil(na1 / kB1Groups))
    double* w;            // [Ra][Rb][NB][na1]: sum over h_b < I_b of V, per next A part
    double* y;            // [Ra][Rb][HB][NA]: the b-runs-out term per I_b
    const double* pa1;    // [HA + 1 + kB1Pad] P(D_a = h), zeros past HA
    const double* fa;     // [HA + 1 + kB1Pad] P(D_a <= h), zeros past HA
    const double* ga;     // [HA + 1 + kB1Pad] P(D_a >= h), zeros past HA
    const double* pb;     // [HB + 1] demand of b
    const double* fb;     // [HB + 1] its CDF
    const double* j;      // [HB][HA][HA] P(h_a, h_b = I_b | I_a, I_b)
    const double* jc;     // [HB][HA][HA] cumulative over h_a
    const double* rev;    // [HA][HB] expected one-day revenue
    const int32_t* xb_order;  // [NB] x_b by digit sum: the final kernels' order
    Ctl* ctl;
    int32_t m, Ra, Rb, HA, HB, na1, nb1, NA, NB, extract;
    int32_t gw;           // stage W: values of the next A part per workgroup
    int32_t cb;           // final stage: orders of b per LDS chunk
    int32_t cbp;          // its LDS row stride in doubles (even, 2 mod 4)
    int32_t lanes_ab;     // 1: the final sweeps use the kernel over lanes of b's orders
                          // where it applies (0: b1_final_kernel everywhere)
    double gamma, cva, cvb;
};
hipError_t launch_backup_b1(const B1Dev& p, int storage_fp32, int extract, hipStream_t s);
// The final kernel over lanes of b's orders: path groups (x_a without X_1) per workgroup,
// and the zeros after a's demand tables (pa1, fa, ga) that its reads at x_1 + k need.
constexpr int kB1Groups = 16;
constexpr int kB1Pad = 48;
hipError_t launch_b1_initial(const B1Dev& p, double* v, hipStream_t s);

// ------------------------------------------------------------------ rollouts
struct SimDev {
    int32_t family, m, L, P, kind, issuing;
    int32_t R0, R1;            // a_max + 1 of product 0 and 1
    int32_t dmax0, dmax1;
    int32_t n_pol, n_roll, warmup, horizon;
    int32_t n_cdf0, n_cdf1, n_lcum;  // entries of the three staged tables
    int64_t start;             // start state index
    uint64_t seed;
    double gamma, rho, mu0, mu1;
    double cvar0, cvar1, cfixed, chold, cshort, cwaste, rev0, rev1;
    const int32_t* table;      // TABLE: action per state
    const int32_t* params;     // heuristics: [n_pol][PVI_POLICY_PARAMS]
    const double* cdf0;        // [P][dmax0 + 1] demand CDF of product 0, summed left to right
    const double* cdf1;        // [dmax1 + 1] demand CDF of product 1 (B)
    const double* lifecum;     // C: [a_max + 1][m], p_1(a) + ... + p_k(a) at a*m + k-1
    double* ret;               // [n_pol * n_roll]
    double* kpi;               // [n_pol * n_roll][3]
    double* pkpi;              // two products: [n_pol * n_roll][2][3], or null
};
hipError_t launch_rollouts(const SimDev& s, hipStream_t st);
// Mean and sample standard deviation of ncol columns of x ([n_pol][n_roll][stride],
// column c at offset c), written to out[p * ostride + ooff + 2 c] and the next slot.
hipError_t launch_column_stats(const double* x, int stride, int ncol, int n_pol, int n_roll,
                               double* out, int ostride, int ooff, hipStream_t st);

// ------------------------------------------------------------------ batched small instances
struct BatchItem {
    int32_t m, R, dmax, tab, xt, ns, nh, stride_a, stride_h, max_sweeps, fixed, fp32;
    double gamma, cvar, thr;
    const double *pmf, *cdf, *tail, *r0;  // scenario-A tables of this instance
    double* v;                            // [ns] returned V (FP64)
    int32_t* pi;                          // [ns] policy
    double* gap;                          // [ns] best - second Q
    double* stats;  // [8]: sweeps fp32, sweeps fp64, span, dmax, dmin, status
};
// The slot kernel (kernels_batch.hip): work group k serves slot k of a table in
// coherent pinned host memory (slot_layout.h) until the host stops it; a request
// already placed in a slot is served before the stop word is honoured.  Instances up
// to kSlotRmax actions; lds_bytes of dynamic LDS per work group.
struct SlotHeader;
struct SlotSync;
constexpr int kSlotRmax = 24;
hipError_t launch_slots(SlotHeader* hdr, SlotSync* sync, const BatchItem* items, int nslots,
                        int threads, size_t lds_bytes, hipStream_t s);
// Work groups of `threads` (64, 128 or 256) of the slot kernel the device keeps
// resident at once (0 if unknown).
int slot_capacity(int threads, size_t lds_bytes);

// launchers (kernels_a.hip)
// LIFO issuing (p.lifo = 1, m >= 2): tiles (O, X_{m-1}..X_2), FP64 accumulation.
hipError_t launch_backup_a_lifo(const ADev& p, int storage_fp32, int extract, hipStream_t s);
hipError_t launch_backup_a(const ADev& p, int storage_fp32, int acc_kahan, int extract,
                           hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Periodic stopping test after sweep i: v[j] = V_{i-j} for j = 0..P (P <= 7);
// partials holds 2 doubles per block of the first kernel.
struct PeriodicArgs {
    const double* v[8];
    int32_t P;
    double gamma, thr;
    int64_t n;
};
constexpr int kPeriodicBlocks = 1024;
hipError_t launch_periodic_check(Ctl* ctl, const PeriodicArgs& a, double* partials,
                                 hipStream_t s);
hipError_t launch_span(Ctl* ctl, const double* partials, int tiles, int storage_fp32,
                       int fixed, double gamma, hipStream_t s);
hipError_t launch_to_f64(const float* v32, double* v64, const Ctl* ctl, int64_t n,
                         hipStream_t s);
hipError_t launch_to_f32(const double* v64, float* v32, double c, int64_t n, hipStream_t s);
hipError_t launch_fill(double* v, double value, int64_t n, hipStream_t s);
// kernels_c.hip
hipError_t launch_backup_c(const CDev& p, int storage_fp32, int extract, hipStream_t s);
// Time the merge kernels of levels 3..m-1 at each block width that fits (4, 8, 12, 16, 32 low
// digits per workgroup) on the handle's own tables, and write the fastest into lb.  With
// order-independent life the top level m-1 is timed as it runs, fused with the final sum.
hipError_t tune_c_merge(const CDev& p, hipStream_t s, int32_t lb[2][10]);
// Span partial slots of a scenario-C sweep whose top merge is fused with the final sum
// (m >= 4, order-independent life): one per workgroup at the narrowest block width, 4
// of the nlo = R^(m-2) low-digit values, for each of the P weekdays.
inline int64_t c_partial_slots(int64_t P, int64_t nlo) { return P * ((nlo + 3) / 4); }
// Most lanes (R x block width) of a workgroup of the fused scenario-C kernels (top merge
// with the final sum; first two merges): two wavefronts per SIMD, so that their per-lane
// sums and offsets fit in registers.
constexpr int kCFusedThreads = 512;
// kernels_b.hip
hipError_t launch_backup_b(const BDev& p, int storage_fp32, int extract, hipStream_t s);

}  // namespace pvi
