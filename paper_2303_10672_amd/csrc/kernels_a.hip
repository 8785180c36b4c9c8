// Scenario A (lead time, FIFO) Bellman backup on gfx950, plus the span reduction
// and the precision-conversion kernels shared by every family.
//
// The backup follows the deterministic-transition update (Methods, "Value
// iteration") with T from Appendix A (FIFO issuing/ageing equation, reward
// equation).  It is organised around two facts about FIFO issuing:
//
//  1. The next state of (O, X_m..X_1) under order a and demand d is
//     (a, O_{L-1}..O_2, O_1 -> X'_m, X'_{m-1}..X'_1), so every outcome of action a
//     lands in one contiguous block of R^(m-1) values, V[a][O][.].  The expected
//     reward does not depend on a except through -c_var*a, so it is a table
//     r0[X_1][sum X] built once on the host.
//  2. Write y = (X_m..X_2).  Demand d <= X_1 leaves y unchanged (only waste);
//     demand d = X_1 + k removes k units from y oldest first, independently of
//     X_1; once k reaches K = sum(y) nothing is left.  So
//         E_a(X_1, y) = F(X_1) V[path_0] + sum_{0<k<K} P(X_1+k) V[path_k]
//                       + P(D >= X_1+K) V[path_K],
//     where path_k is y depleted by k units.  For a fixed (X_m..X_3) the paths of
//     all X_2 lie on one descending list of (m-1)(R-1)+1 points at most, so a
//     workgroup stages that list for every action in LDS and each lane (one
//     state (X_2, X_1)) walks its own suffix of it.  Per state and action this
//     is K+1 <= d_max+1 multiply-adds instead of d_max+1 gathers.
//
// Workgroup = one tile (O, X_m..X_3) of R*R states (X_2, X_1); lanes = states.
// Ties in the max go to the lowest action.  No atomics: every reduction is a
// fixed tree, so reruns are bit-identical.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "device_common.h"
#include "pvi_internal.h"

namespace pvi {

// Offset inside a next-state block of point j of a tile's descending path list.
// The list is [col_{m-1} (Y_{m-1} points), ..., col_2 (Y_2 points), row (r2 points)]
// where Y_i = X_{i+1} are the tile's fixed digits and col_i[t] has digit i = t,
// the higher digits of the tile and zeros below.
__device__ __forceinline__ int path_offset(int j, const int* Y, int m, const int* pw) {
    int off = 0;
    for (int i = m - 1; i >= 2; --i) {
        if (j < Y[i]) return off + j * pw[i - 1];
        j -= Y[i];
        off += Y[i] * pw[i - 1];
    }
    return off + j;
}

template <typename VT>
struct VecLoad;
template <>
struct VecLoad<float> {
    using V = float4;
    static constexpr int W = 4;
};
template <>
struct VecLoad<double> {
    using V = double2;
    static constexpr int W = 2;
};

template <typename VT, int W>
__device__ __forceinline__ VT lane_of(const typename VecLoad<VT>::V& v, int i);
template <>
__device__ __forceinline__ float lane_of<float, 4>(const float4& v, int i) {
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}
template <>
__device__ __forceinline__ double lane_of<double, 2>(const double2& v, int i) {
    return i == 0 ? v.x : v.y;
}

// Accumulator over outcomes: FP64 multiply-add, or FP32 with Kahan compensation.
template <typename VT, bool KAHAN>
struct Acc {
    using W = double;
    double s = 0.0;
    __device__ __forceinline__ void add(double w, VT u) { s = fma(w, (double)u, s); }
    __device__ __forceinline__ double value() const { return s; }
};
template <>
struct Acc<float, true> {
    using W = float;
    float s = 0.f, c = 0.f;
    __device__ __forceinline__ void add(float w, float u) {
        const float y = fmaf(w, u, -c);
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ double value() const { return (double)s - (double)c; }
};

// VT: storage type of V (float = centred FP32, double = FP64).
// KAHAN: FP32 compensated accumulation (only with VT = float); otherwise FP64.
// J: states (consecutive X_1) per lane.  Lanes with the same X_2 read the same
//    staged values, so each value read from LDS feeds J multiply-adds; this keeps
//    the LDS return path from limiting the kernel.
// EXTRACT: write policy and Q gap instead of V (FP64 only).
template <typename VT, bool KAHAN, int RMAX, int J, bool EXTRACT>
__global__ __launch_bounds__(512) void backup_a_kernel(ADev p) {
    extern __shared__ __align__(16) unsigned char smem[];
    Ctl* ctl = p.ctl;
    if (!EXTRACT && ctl->stop) return;
    constexpr int W = VecLoad<VT>::W;
    using VV = typename VecLoad<VT>::V;
    using AW = typename Acc<VT, KAHAN>::W;

    const int R = p.R, m = p.m, tid = threadIdx.x, bs = blockDim.x;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int h = tile / p.nz;
    int Y[9];
    int b = 0;
    {
        int t = tile - h * p.nz;
        for (int i = 2; i <= m - 1; ++i) {
            Y[i] = t % R;
            t /= R;
            b += Y[i];
        }
    }
    const int lp = b + p.r2;

    VT* S = reinterpret_cast<VT*>(smem);
    // RMAX is a multiple of 8, so the staged block ends on a 32-byte boundary.
    double* sP = reinterpret_cast<double*>(smem + sizeof(VT) * (size_t)lp * RMAX);
    double* sF = sP + p.tab;
    double* sG = sF + p.tab;
    double* red = sG + p.tab;

    for (int i = tid; i < p.tab; i += bs) {
        sP[i] = p.pmf[i];
        sF[i] = p.cdf[i];
        sG[i] = p.tail[i];
    }
    const VT* vin = reinterpret_cast<const VT*>(p.v_in);
    const int64_t hbase = (int64_t)h * p.stride_h;
    for (int idx = tid; idx < lp * RMAX; idx += bs) {
        const int a = idx / lp, j = idx - a * lp;
        VT v = VT(0);
        if (a < R) v = vin[(int64_t)a * p.stride_a + hbase + path_offset(j, Y, m, p.pow_y)];
        S[j * RMAX + a] = v;
    }
    __syncthreads();

    const int G = (R + J - 1) / J;
    const int ns_tile = p.r2 * R;
    const bool active = tid < p.r2 * G;
    const int X2 = active ? tid / G : 0;
    const int x1_0 = active ? (tid - X2 * G) * J : 0;
    double dmx = -DBL_MAX, dmn = DBL_MAX, vmx = -DBL_MAX, vmn = DBL_MAX;
    if (active) {
        const int N = b + X2;
        const int kmax = N == 0 ? 0 : max(0, min(N, p.dmax - x1_0));
        Acc<VT, KAHAN> acc[J][RMAX];
        for (int k = 0; k <= kmax; ++k) {
            AW w[J];
#pragma unroll
            for (int i = 0; i < J; ++i) {
                const int X1 = x1_0 + i;
                // demand <= X_1 keeps y; X_1 + k removes k units; the last point
                // collects every demand that empties y (tables are zero past d_max)
                const double wd = N == 0 ? (k == 0 ? 1.0 : 0.0)
                                  : k == 0 ? sF[min(X1, p.dmax)]
                                  : k == N ? sG[X1 + N]
                                           : sP[X1 + k];
                w[i] = (AW)wd;
            }
            const VV* row = reinterpret_cast<const VV*>(S + (N - k) * RMAX);
#pragma unroll
            for (int q = 0; q < RMAX / W; ++q) {
                const VV u = row[q];
#pragma unroll
                for (int e = 0; e < W; ++e) {
                    const VT ue = lane_of<VT, W>(u, e);
#pragma unroll
                    for (int i = 0; i < J; ++i) acc[i][q * W + e].add(w[i], ue);
                }
            }
        }
        const double mu = (!EXTRACT && sizeof(VT) == 4) ? ctl->mu : 0.0;
#pragma unroll
        for (int i = 0; i < J; ++i) {
            const int X1 = x1_0 + i;
            if (X1 >= R) continue;
            double best = -DBL_MAX, second = -DBL_MAX;
            int arg = 0;
#pragma unroll
            for (int a = 0; a < RMAX; ++a) {
                if (a < R) {
                    const double q = -p.cvar * a + p.gamma * acc[i][a].value();
                    if (q > best) {
                        second = best;
                        best = q;
                        arg = a;
                    } else if (q > second) {
                        second = q;
                    }
                }
            }
            const int64_t s_idx = (int64_t)tile * ns_tile + X2 * R + X1;
            if (EXTRACT) {
                p.pi[s_idx] = arg;
                p.gap[s_idx] = R > 1 ? best - second : INFINITY;
            } else {
                const double r0 = p.r0[X1 * p.xt + X1 + X2 + b];
                const VT o = (VT)(r0 - mu + best);
                reinterpret_cast<VT*>(p.v_out)[s_idx] = o;
                const double out = (double)o, dv = out - (double)vin[s_idx];
                dmx = fmax(dmx, dv);
                dmn = fmin(dmn, dv);
                vmx = fmax(vmx, out);
                vmn = fmin(vmn, out);
            }
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

// Single-workgroup reduction of the per-tile partials and the stopping rule.
__global__ __launch_bounds__(1024) void span_kernel(Ctl* ctl, const double* partials,
                                                    int tiles, int fp32, int fixed,
                                                    double gamma) {
    __shared__ double red[4 * 16];
    if (ctl->stop) return;
    double a0 = -DBL_MAX, a1 = DBL_MAX, a2 = -DBL_MAX, a3 = DBL_MAX;
    for (int i = threadIdx.x; i < tiles; i += blockDim.x) {
        a0 = fmax(a0, partials[4 * i + 0]);
        a1 = fmin(a1, partials[4 * i + 1]);
        a2 = fmax(a2, partials[4 * i + 2]);
        a3 = fmin(a3, partials[4 * i + 3]);
    }
    block_reduce4(a0, a1, a2, a3, red);
    if (threadIdx.x != 0) return;
    double dmax = a0, dmin = a1;
    if (fp32) {
        // V = c + v: V_new - V = ((gamma-1) c + mu) + (v_new - v)
        const double shift = (gamma - 1.0) * ctl->c + ctl->mu;
        dmax += shift;
        dmin += shift;
        ctl->c = gamma * ctl->c + ctl->mu;
        ctl->mu += 0.5 * (a2 + a3);
    }
    const double span = dmax - dmin;
    ctl->dmax = dmax;
    ctl->dmin = dmin;
    ctl->span = span;
    ctl->sweeps += 1;
    if (fixed) return;
    if (fp32) {
        const double vabs = fmax(fabs(a2), fabs(a3));
        ctl->vabs = vabs;
        if (span < ctl->best_span * 0.999) {
            ctl->best_span = span;
            ctl->stall = 0;
        } else {
            ctl->stall += 1;
        }
        if (span < ctl->thr || span <= ctl->floor32 * vabs || ctl->stall >= 3) {
            ctl->stop = 1;
            ctl->stop_sweep = ctl->sweeps;
        }
    } else if (span < ctl->thr) {
        ctl->stop = 1;
        ctl->stop_sweep = ctl->sweeps;
    }
}

__global__ void to_f64_kernel(const float* v32, double* v64, const Ctl* ctl, int64_t n) {
    const double c = ctl->c;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        v64[i] = c + (double)v32[i];
}

__global__ void fill_kernel(double* v, double value, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        v[i] = value;
}

__global__ void to_f32_kernel(const double* v64, float* v32, double c, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        v32[i] = (float)(v64[i] - c);
}

// ------------------------------------------------------------------ launchers

template <typename VT, bool KAHAN, bool EXTRACT, int RMAX>
static hipError_t launch_a_r(const ADev& p, hipStream_t s) {
    // states per lane: enough multiply-adds per LDS value to keep VALU busy
    constexpr int J = KAHAN ? 2 : (RMAX <= 24 ? 4 : 3);
    const int lp_max = (p.m >= 2 ? (p.m - 2) * (p.R - 1) : 0) + p.r2;
    size_t bytes = sizeof(VT) * (size_t)lp_max * RMAX;
    bytes += sizeof(double) * (3 * (size_t)p.tab + 64);
    if (bytes > 65536) return hipErrorInvalidConfiguration;  // beyond the default LDS limit
    if (p.tab < p.R + J + lp_max || p.tab < p.dmax + 2 + J) return hipErrorInvalidValue;
    const int lanes = p.r2 * ((p.R + J - 1) / J);
    const int threads = ((lanes + 63) / 64) * 64;
    if (threads > 512) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((backup_a_kernel<VT, KAHAN, RMAX, J, EXTRACT>), dim3(p.tiles),
                       dim3(threads), bytes, s, p);
    return hipGetLastError();
}

template <typename VT, bool KAHAN, bool EXTRACT>
static hipError_t launch_a_t(const ADev& p, hipStream_t s) {
    if (p.R <= 8) return launch_a_r<VT, KAHAN, EXTRACT, 8>(p, s);
    if (p.R <= 16) return launch_a_r<VT, KAHAN, EXTRACT, 16>(p, s);
    if (p.R <= 24) return launch_a_r<VT, KAHAN, EXTRACT, 24>(p, s);
    if (p.R <= 32) return launch_a_r<VT, KAHAN, EXTRACT, 32>(p, s);
    return hipErrorInvalidValue;
}

hipError_t launch_backup_a(const ADev& p, int storage_fp32, int acc_kahan, int extract,
                           hipStream_t s) {
    if (extract) return launch_a_t<double, false, true>(p, s);
    if (storage_fp32) {
        if (acc_kahan) return launch_a_t<float, true, false>(p, s);
        return launch_a_t<float, false, false>(p, s);
    }
    return launch_a_t<double, false, false>(p, s);
}

hipError_t launch_span(Ctl* ctl, const double* partials, int tiles, int storage_fp32,
                       int fixed, double gamma, hipStream_t s) {
    hipLaunchKernelGGL(span_kernel, dim3(1), dim3(1024), 0, s, ctl, partials, tiles,
                       storage_fp32, fixed, gamma);
    return hipGetLastError();
}

hipError_t launch_to_f64(const float* v32, double* v64, const Ctl* ctl, int64_t n,
                         hipStream_t s) {
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(to_f64_kernel, dim3(blocks), dim3(256), 0, s, v32, v64, ctl, n);
    return hipGetLastError();
}

hipError_t launch_to_f32(const double* v64, float* v32, double c, int64_t n,
                         hipStream_t s) {
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(to_f32_kernel, dim3(blocks), dim3(256), 0, s, v64, v32, c, n);
    return hipGetLastError();
}

hipError_t launch_fill(double* v, double value, int64_t n, hipStream_t s) {
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(256), 0, s, v, value, n);
    return hipGetLastError();
}

}  // namespace pvi
