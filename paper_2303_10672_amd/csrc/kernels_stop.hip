// The periodic stopping test of Appendix C, for MDPs whose dynamics repeat with
// period P (scenario C's weekdays).  The paper sums the last P increments
// gamma^-(i-j-1) (V_{i-j} - V_{i-j-1}); multiplied by gamma^(i-1) that is
//   D(s) = sum_{j=0}^{P-1} gamma^j (V_{i-j}(s) - V_{i-j-1}(s)),
// and the test  max D - min D <= 2 eps min(|max D|, |min D|)  is unchanged by the
// factor.  Two launches per sweep: per-block max/min of D over a grid-stride loop,
// then one workgroup that reduces them and sets the stop flag.  Both return at once
// when the flag is already set, like every launch of the sweep loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>

#include "device_common.h"
#include "pvi_internal.h"

namespace pvi {

__global__ __launch_bounds__(256) void periodic_partial_kernel(const Ctl* ctl, PeriodicArgs a,
                                                               double* partials) {
    __shared__ double red[64];
    if (ctl->stop) return;
    double dmx = -DBL_MAX, dmn = DBL_MAX;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < a.n;
         s += (int64_t)gridDim.x * blockDim.x) {
        double D = 0.0, w = 1.0;
        for (int j = 0; j < a.P; ++j) {
            D = fma(w, a.v[j][s] - a.v[j + 1][s], D);
            w *= a.gamma;
        }
        dmx = fmax(dmx, D);
        dmn = fmin(dmn, D);
    }
    double c = dmx, d = dmn;  // block_reduce4 reduces four values; two are used
    block_reduce4(dmx, dmn, c, d, red);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = dmx;
        partials[2 * blockIdx.x + 1] = dmn;
    }
}

__global__ __launch_bounds__(1024) void periodic_reduce_kernel(Ctl* ctl, const double* partials,
                                                               int nblocks, double thr) {
    __shared__ double red[64];
    if (ctl->stop) return;
    double dmx = -DBL_MAX, dmn = DBL_MAX;
    for (int i = threadIdx.x; i < nblocks; i += blockDim.x) {
        dmx = fmax(dmx, partials[2 * i]);
        dmn = fmin(dmn, partials[2 * i + 1]);
    }
    double c = dmx, d = dmn;
    block_reduce4(dmx, dmn, c, d, red);
    if (threadIdx.x == 0 && dmx - dmn <= 2.0 * thr * fmin(fabs(dmx), fabs(dmn))) {
        ctl->stop = 1;
        ctl->stop_sweep = ctl->sweeps;
    }
}

hipError_t launch_periodic_check(Ctl* ctl, const PeriodicArgs& a, double* partials,
                                 hipStream_t s) {
    if (a.P < 1 || a.P > 7 || a.n < 1) return hipErrorInvalidValue;
    const int blocks = (int)std::min<int64_t>((a.n + 255) / 256, kPeriodicBlocks);
    hipLaunchKernelGGL(periodic_partial_kernel, dim3(blocks), dim3(256), 0, s, ctl, a, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // one wavefront per 64 partials, at most 1024 threads (max and min are exact)
    const int threads = blocks >= 1024 ? 1024 : blocks <= 64 ? 64 : (blocks + 63) / 64 * 64;
    hipLaunchKernelGGL(periodic_reduce_kernel, dim3(1), dim3(threads), 0, s, ctl, partials,
                       blocks, a.thr);
    return hipGetLastError();
}

}  // namespace pvi
