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

    int64_t logical_per_sweep = 0;
    int64_t executed_per_sweep = 0;

    // device state (allocated on the first solve)
    struct Dev {
        bool ready = false;
        int device = -1;
        hipStream_t own = nullptr;
        double* v64[2] = {nullptr, nullptr};
        float* v32[2] = {nullptr, nullptr};
        int32_t* pi = nullptr;
        double* gap = nullptr;
        double* partials = nullptr;
        pvi::Ctl* ctl = nullptr;
        pvi::Ctl* h_ctl = nullptr;  // pinned host mirror
        double *pmf = nullptr, *cdf = nullptr, *tail = nullptr, *r0 = nullptr;
        int tiles = 0;
        size_t bytes = 0;
        std::vector<hipEvent_t> ev;
    } dev;

    // results of the last solve
    int have_result = 0;
    int ret_buf = 0;  // v64 buffer holding V
    std::mutex mu;
};

namespace pvi {
pvi_status ensure_device(pvi_mdp* p);
void free_device(pvi_mdp* p);
size_t device_bytes(const pvi_mdp* p);
pvi::ADev make_adev(const pvi_mdp* p);
}  // namespace pvi
