// Scenario A backup with LIFO issuing (Appendix A, LIFO issuing/ageing equation).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>

#include "device_common.h"
#include "pvi_internal.h"

namespace pvi {

// Scenario A with LIFO issuing (Appendix A, LIFO issuing/ageing equation).  The
// youngest units go first, so demand d removes min(d, K) units from
// y = (X_m..X_2) youngest first (K = X_2 + ... + X_m); only what is left of the
// demand reaches X_1, whose remainder expires.  The next state depends on y and
// d but not on X_1, so the expectation E_a(O, y), the best action and the Q gap
// are shared by the R states (O, y, X_1), which differ only in the expected
// reward r0[X_1][K] (host table).  Read backwards, the depletion path of y is a
// list L with L[0] = nothing left and L[i] = the i units issued last, so
//   E_a = sum_{i=1}^{K} P(K - i) L_a[i] + P(D >= K) L_a[0].
// Workgroup = tile (O, X_{m-1}..X_2); its R values of X_m = t share one list of
// b + R points (b = X_2 + ... + X_{m-1}): points 1..b rebuild X_2 first, then
// X_3, ..., X_{m-1}; point b + t is (X_m = t, the rest full).  Lanes (t, a) form
// E_a for K = b + t; one lane per t takes the max (ties to the lowest action);
// lanes (t, X_1) write the states.  FP64 accumulation for every storage type.
template <typename VT, bool EXTRACT>
__global__ __launch_bounds__(1024) void backup_a_lifo_kernel(ADev p) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[64];
    Ctl* ctl = p.ctl;
    if (!EXTRACT && ctl->stop) return;
    const int R = p.R, m = p.m, tid = threadIdx.x, nt = blockDim.x;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int h = tile / p.nz, z = tile - h * p.nz;  // z = (X_{m-1}..X_2), X_2 fastest
    int Y[10];  // Y[j] = X_j, j = 2 .. m-1
    int b = 0;
    {
        int t = z;
        for (int j = 2; j <= m - 1; ++j) {
            Y[j] = t % R;
            t /= R;
            b += Y[j];
        }
    }
    const int lp = b + R;
    double* L = reinterpret_cast<double*>(smem);  // [lp][R]
    double* sq = L + (size_t)p.lmax * R;           // [R][R] Q(t, a)
    double* sP = sq + (size_t)R * R;
    double* sG = sP + p.tab;
    double* sM = sG + p.tab;  // [R] best Q per t
    double* sS = sM + R;      // [R] second best
    int* sA = reinterpret_cast<int*>(sS + R);  // [R] argmax
    for (int i = tid; i < p.tab; i += nt) {
        sP[i] = p.pmf[i];
        sG[i] = p.tail[i];
    }
    const VT* vin = reinterpret_cast<const VT*>(p.v_in);
    const int64_t hbase = (int64_t)h * p.stride_h;
    for (int k = tid; k < lp * R; k += nt) {
        const int i = k / R, a = k - i * R;
        int off;
        if (i > b) {
            off = (i - b) * p.pow_y[m - 2] + z;  // X_m = i - b, the rest full
        } else {
            off = 0;  // i units: X_2 filled first, then X_3, ...
            int left = i;
            for (int j = 2; j <= m - 1; ++j) {
                const int f = min(left, Y[j]);
                off += f * p.pow_y[j - 2];
                left -= f;
            }
        }
        L[i * R + a] = (double)vin[hbase + (int64_t)a * p.stride_a + off];
    }
    __syncthreads();
    for (int k = tid; k < R * R; k += nt) {
        const int t = k / R, a = k - t * R, K = b + t;
        double e = sG[K] * L[a];
        for (int i = 1; i <= K; ++i) e = fma(sP[K - i], L[i * R + a], e);
        sq[k] = fma(p.gamma, e, -p.cvar * a);
    }
    __syncthreads();
    if (tid < R) {
        double best = -DBL_MAX, second = -DBL_MAX;
        int arg = 0;
        for (int a = 0; a < R; ++a) {
            const double q = sq[tid * R + a];
            if (q > best) {
                second = best;
                best = q;
                arg = a;
            } else if (q > second) {
                second = q;
            }
        }
        sM[tid] = best;
        sS[tid] = second;
        sA[tid] = arg;
    }
    __syncthreads();
    const int64_t base = (int64_t)h * p.stride_h * R + (int64_t)z * R;
    const int64_t tstride = (int64_t)p.pow_y[m - 2] * R;  // R^(m-1): one step of X_m
    const double mu = (!EXTRACT && sizeof(VT) == 4) ? ctl->mu : 0.0;
    double dmx = -DBL_MAX, dmn = DBL_MAX, vmx = -DBL_MAX, vmn = DBL_MAX;
    for (int k = tid; k < R * R; k += nt) {
        const int t = k / R, x1 = k - t * R;
        const int64_t s_idx = base + t * tstride + x1;
        if (EXTRACT) {
            p.pi[s_idx] = sA[t];
            p.gap[s_idx] = R > 1 ? sM[t] - sS[t] : INFINITY;
        } else {
            const VT o = (VT)(p.r0[x1 * p.xt + b + t] - mu + sM[t]);
            reinterpret_cast<VT*>(p.v_out)[s_idx] = o;
            const double out = (double)o, dv = out - (double)vin[s_idx];
            dmx = fmax(dmx, dv);
            dmn = fmin(dmn, dv);
            vmx = fmax(vmx, out);
            vmn = fmin(vmn, out);
        }
    }
    if (EXTRACT) return;
    block_reduce4(dmx, dmn, vmx, vmn, red);
    if (tid == 0) {
        double* pp = p.partials + 4 * (size_t)tile;
        pp[0] = dmx;
        pp[1] = dmn;
        pp[2] = vmx;
        pp[3] = vmn;
    }
}

static size_t a_lifo_lds_bytes(const ADev& p) {
    return sizeof(double) * ((size_t)p.lmax * p.R + (size_t)p.R * p.R + 2 * (size_t)p.tab +
                             2 * (size_t)p.R) +
           sizeof(int) * (size_t)p.R;
}

hipError_t launch_backup_a_lifo(const ADev& p, int storage_fp32, int extract, hipStream_t s) {
    // tiles (O, X_{m-1}..X_2); lanes over (X_m, action) and (X_m, X_1)
    if (p.m < 2 || p.R > 32 || p.tiles < 1) return hipErrorInvalidConfiguration;
    const size_t bytes = a_lifo_lds_bytes(p);
    if (bytes > 65536) return hipErrorInvalidConfiguration;
    if (p.tab < p.lmax + 1 || p.lmax < (p.m - 2) * (p.R - 1) + p.R)
        return hipErrorInvalidValue;
    const int threads = std::min(1024, ((p.R * p.R + 63) / 64) * 64);
    if (extract)
        hipLaunchKernelGGL((backup_a_lifo_kernel<double, true>), dim3(p.tiles), dim3(threads),
                           bytes, s, p);
    else if (storage_fp32)
        hipLaunchKernelGGL((backup_a_lifo_kernel<float, false>), dim3(p.tiles), dim3(threads),
                           bytes, s, p);
    else
        hipLaunchKernelGGL((backup_a_lifo_kernel<double, false>), dim3(p.tiles), dim3(threads),
                           bytes, s, p);
    return hipGetLastError();
}

}  // namespace pvi
