// Batched value iteration of many small scenario-A instances in one launch.
//
// One workgroup solves one instance completely: both value tables live in LDS,
// the workgroup sweeps (deterministic-transition update of Methods, "Value
// iteration"; T from Appendix A), reduces max/min of V_new - V itself, applies
// the span stopping rule, and finally extracts the greedy policy with one more
// FP64 backup.  The FP32 schedule keeps V in LDS as centred FP32 (V = c + v)
// until the span reaches the FP32 floor, then converts to FP64 and polishes to
// the threshold.  Every instance has its own sizes, costs and tables, so a batch
// may mix instances; each workgroup's arithmetic depends only on its own instance,
// which makes results independent of the batch they ran in.  The sweep loop is
// bounded by max_sweeps, so every workgroup exits.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "device_common.h"
#include "pvi_internal.h"

namespace pvi {

struct BatchShared {
    double dmax, dmin, vmax, vmin;
    double c, mu, best_span;
    int stop, stall;
};

// One synchronous sweep src -> dst over all states (or the policy extraction).
// Returns through sh the max/min of dst - src and of dst.
template <typename VT, int RMAX, bool EXTRACT>
__device__ void batch_sweep(const BatchItem& it, const VT* src, VT* dst, const double* sP,
                            const double* sF, const double* sG, const double* sR0, double mu,
                            double* red, BatchShared* sh) {
    const int R = it.R, m = it.m;
    double dmx = -DBL_MAX, dmn = DBL_MAX, vmx = -DBL_MAX, vmn = DBL_MAX;
    const int nx = it.ns / it.nh;  // R^m stock vectors per in-transit vector
    for (int s = threadIdx.x; s < it.ns; s += blockDim.x) {
        const int h = s / nx;
        int x = s - h * nx;
        const int X1 = x % R;
        x /= R;
        int Y[9];  // Y[j] = X_{j+1}
        int K = 0;
        for (int j = 1; j <= m - 1; ++j) {
            Y[j] = x % R;
            x /= R;
            K += Y[j];
        }
        const int kmax = K == 0 ? 0 : max(0, min(K, it.dmax - X1));
        double acc[RMAX];
#pragma unroll
        for (int a = 0; a < RMAX; ++a) acc[a] = 0.0;
        const int base = h * it.stride_h;
        for (int k = 0; k <= kmax; ++k) {
            // y depleted by k units, oldest first
            int r = k, off = 0, pw = 1;
            for (int j = 1; j <= m - 1; ++j) {
                const int take = min(r, Y[j]);
                r -= take;
                off += (Y[j] - take) * pw;
                pw *= R;
            }
            const double w = K == 0 ? 1.0 : k == 0 ? sF[min(X1, it.dmax)] : k == K ? sG[X1 + K]
                                                                                 : sP[X1 + k];
            const VT* col = src + base + off;
#pragma unroll
            for (int a = 0; a < RMAX; ++a)
                if (a < R) acc[a] = fma(w, (double)col[a * it.stride_a], acc[a]);
        }
        double best = -DBL_MAX, second = -DBL_MAX;
        int arg = 0;
#pragma unroll
        for (int a = 0; a < RMAX; ++a) {
            if (a < R) {
                const double q = -it.cvar * a + it.gamma * acc[a];
                if (q > best) {
                    second = best;
                    best = q;
                    arg = a;
                } else if (q > second) {
                    second = q;
                }
            }
        }
        if (EXTRACT) {
            it.pi[s] = arg;
            it.gap[s] = R > 1 ? best - second : INFINITY;
        } else {
            const int xtot = X1 + K;
            const VT o = (VT)(sR0[X1 * it.xt + xtot] - mu + best);
            dst[s] = o;
            const double out = (double)o, dv = out - (double)src[s];
            dmx = fmax(dmx, dv);
            dmn = fmin(dmn, dv);
            vmx = fmax(vmx, out);
            vmn = fmin(vmn, out);
        }
    }
    if (EXTRACT) return;
    block_reduce4(dmx, dmn, vmx, vmn, red);
    if (threadIdx.x == 0) {
        sh->dmax = dmx;
        sh->dmin = dmn;
        sh->vmax = vmx;
        sh->vmin = vmn;
    }
    __syncthreads();
}

template <int RMAX>
__global__ __launch_bounds__(256) void batch_solve_kernel(const BatchItem* items) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[64];
    __shared__ BatchShared sh;
    const BatchItem it = items[blockIdx.x];
    double* V0 = reinterpret_cast<double*>(smem);
    double* V1 = V0 + it.ns;
    double* sP = V1 + it.ns;
    double* sF = sP + it.tab;
    double* sG = sF + it.tab;
    double* sR0 = sG + it.tab;
    for (int i = threadIdx.x; i < it.tab; i += blockDim.x) {
        sP[i] = it.pmf[i];
        sF[i] = it.cdf[i];
        sG[i] = it.tail[i];
    }
    for (int i = threadIdx.x; i < it.R * it.xt; i += blockDim.x) sR0[i] = it.r0[i];
    const double g = it.gamma;
    int sweeps32 = 0, sweeps64 = 0, converged = 0;
    double span = INFINITY, dmax = 0.0, dmin = 0.0;
    if (it.fp32) {
        // centred FP32 storage: V = c + v, c in FP64
        float* v0 = reinterpret_cast<float*>(V0);
        float* v1 = reinterpret_cast<float*>(V1);
        for (int i = threadIdx.x; i < it.ns; i += blockDim.x) v0[i] = 0.f;
        if (threadIdx.x == 0) {
            sh.c = 0.0;
            sh.mu = 0.0;
            sh.best_span = INFINITY;
            sh.stop = 0;
            sh.stall = 0;
        }
        __syncthreads();
        const int limit = it.fixed > 0 ? it.fixed : it.max_sweeps;
        for (int n = 0; n < limit; ++n) {
            float* src = (n & 1) ? v1 : v0;
            float* dst = (n & 1) ? v0 : v1;
            batch_sweep<float, RMAX, false>(it, src, dst, sP, sF, sG, sR0, sh.mu, red, &sh);
            ++sweeps32;
            if (threadIdx.x == 0) {
                const double shift = (g - 1.0) * sh.c + sh.mu;
                dmax = sh.dmax + shift;
                dmin = sh.dmin + shift;
                span = dmax - dmin;
                sh.c = g * sh.c + sh.mu;
                sh.mu += 0.5 * (sh.vmax + sh.vmin);
                const double vabs = fmax(fabs(sh.vmax), fabs(sh.vmin));
                if (span < sh.best_span * 0.999) {
                    sh.best_span = span;
                    sh.stall = 0;
                } else {
                    sh.stall += 1;
                }
                if (it.fixed <= 0 &&
                    (span < it.thr || span <= 4.0 * 1.1920928955078125e-07 * vabs || sh.stall >= 3))
                    sh.stop = 1;
                sh.dmax = dmax;
                sh.dmin = dmin;
            }
            __syncthreads();
            if (sh.stop) break;
        }
        // to FP64 in place order: read the FP32 result, write FP64 into the other table
        const float* res = (sweeps32 & 1) ? v1 : v0;
        double* out = (sweeps32 & 1) ? V0 : V1;
        // res and out must not overlap: res is float* into one table, out the other
        const double c = sh.c;
        for (int i = threadIdx.x; i < it.ns; i += blockDim.x) out[i] = c + (double)res[i];
        __syncthreads();
        if (out != V0) {
            for (int i = threadIdx.x; i < it.ns; i += blockDim.x) V0[i] = V1[i];
            __syncthreads();
        }
        dmax = sh.dmax;
        dmin = sh.dmin;
    } else {
        for (int i = threadIdx.x; i < it.ns; i += blockDim.x) V0[i] = 0.0;
        __syncthreads();
    }
    // FP64 phase (the whole solve for FP64, the polish for the FP32 schedule)
    int cur = 0;
    if (!(it.fp32 && it.fixed > 0)) {
        const int limit = (!it.fp32 && it.fixed > 0) ? it.fixed : it.max_sweeps;
        for (int n = 0; n < limit; ++n) {
            double* src = cur ? V1 : V0;
            double* dst = cur ? V0 : V1;
            batch_sweep<double, RMAX, false>(it, src, dst, sP, sF, sG, sR0, 0.0, red, &sh);
            cur ^= 1;
            ++sweeps64;
            dmax = sh.dmax;
            dmin = sh.dmin;
            span = dmax - dmin;
            if (it.fixed <= 0 && span < it.thr) {
                converged = 1;
                break;
            }
        }
        if (it.fixed > 0) converged = 1;
    } else {
        converged = 1;
    }
    double* Vret = cur ? V1 : V0;
    batch_sweep<double, RMAX, true>(it, Vret, nullptr, sP, sF, sG, sR0, 0.0, red, &sh);
    for (int i = threadIdx.x; i < it.ns; i += blockDim.x) it.v[i] = Vret[i];
    if (threadIdx.x == 0) {
        it.stats[0] = sweeps32;
        it.stats[1] = sweeps64;
        it.stats[2] = span;
        it.stats[3] = dmax;
        it.stats[4] = dmin;
        it.stats[5] = converged ? 0.0 : (double)PVI_E_NOT_CONVERGED;
    }
}

hipError_t launch_batch(const BatchItem* d_items, int n, size_t lds_bytes, int rmax,
                        hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (lds_bytes > 65536) return hipErrorInvalidConfiguration;
    if (rmax <= 8)
        hipLaunchKernelGGL((batch_solve_kernel<8>), dim3(n), dim3(256), lds_bytes, s, d_items);
    else if (rmax <= 16)
        hipLaunchKernelGGL((batch_solve_kernel<16>), dim3(n), dim3(256), lds_bytes, s, d_items);
    else if (rmax <= 24)
        hipLaunchKernelGGL((batch_solve_kernel<24>), dim3(n), dim3(256), lds_bytes, s, d_items);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace pvi
