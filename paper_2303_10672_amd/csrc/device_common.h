// Device helpers shared by the kernel files (header-only, no relocatable code).
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "pvi_internal.h"

namespace pvi {

__device__ __forceinline__ int xcd_remap(int bid, int nb) {
    // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous range of tiles so the V blocks a range touches stay in one L2.
    const int q = nb >> 3, r = nb & 7, x = bid & 7, l = bid >> 3;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + l;
}

__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Block-wide reduction of 4 values (max, min, max, min); result valid in thread 0.
__device__ inline void block_reduce4(double& a, double& b, double& c, double& d, double* red) {
    a = wave_max(a);
    b = wave_min(b);
    c = wave_max(c);
    d = wave_min(d);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if (lane == 0) {
        red[4 * w + 0] = a;
        red[4 * w + 1] = b;
        red[4 * w + 2] = c;
        red[4 * w + 3] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < nw; ++i) {
            a = fmax(a, red[4 * i + 0]);
            b = fmin(b, red[4 * i + 1]);
            c = fmax(c, red[4 * i + 2]);
            d = fmin(d, red[4 * i + 3]);
        }
    }
}

// Stopping rule applied to the reduced (max dv, min dv, max v', min v') of one sweep,
// on a copy of the control block that the caller writes back.
// With FP32 storage (V = c + v) it also moves the centring: c <- gamma c + mu and
// mu <- mu + mid(v').  Called by one thread after the whole sweep is reduced.
__device__ inline void span_update(Ctl& ctl, double a0, double a1, double a2, double a3,
                                   int fp32, int fixed, double gamma) {
    double dmax = a0, dmin = a1;
    if (fp32) {
        const double shift = (gamma - 1.0) * ctl.c + ctl.mu;
        dmax += shift;
        dmin += shift;
        ctl.c = gamma * ctl.c + ctl.mu;
        ctl.mu += 0.5 * (a2 + a3);
    }
    const double span = dmax - dmin;
    // stopping criterion: the span (rule 0) or max |V_new - V| (rule 1)
    // (the periodic rule, 2, is decided by its own kernels after this one)
    const double crit = ctl.rule == 1   ? fmax(fabs(dmax), fabs(dmin))
                        : ctl.rule == 2 ? INFINITY
                                         : span;
    ctl.dmax = dmax;
    ctl.dmin = dmin;
    ctl.span = span;
    ctl.sweeps += 1;
    if (fixed) return;
    if (fp32) {
        const double vabs = fmax(fabs(a2), fabs(a3));
        ctl.vabs = vabs;
        if (span < ctl.best_span * 0.999) {
            ctl.best_span = span;
            ctl.stall = 0;
        } else {
            ctl.stall += 1;
        }
        // the FP32 phase hands over to FP64 at the FP32 floor (span based for
        // either rule) or when the rule itself is met
        if (crit < ctl.thr || span <= ctl.floor32 * vabs || ctl.stall >= 3) {
            ctl.stop = 1;
            ctl.stop_sweep = ctl.sweeps;
        }
    } else if (crit < ctl.thr) {
        ctl.stop = 1;
        ctl.stop_sweep = ctl.sweeps;
    }
}

}  // namespace pvi
