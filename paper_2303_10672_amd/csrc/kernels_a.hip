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

template <typename VT>
__device__ __forceinline__ typename VecLoad<VT>::V make_vec(const VT* v);
template <>
__device__ __forceinline__ float4 make_vec<float>(const float* v) {
    return make_float4(v[0], v[1], v[2], v[3]);
}
template <>
__device__ __forceinline__ double2 make_vec<double>(const double* v) {
    return make_double2(v[0], v[1]);
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
// Lanes: (X_2, group of J consecutive X_1, half of the actions).  Lanes with the
//   same X_2 read the same staged values, so each LDS value feeds J multiply-adds;
//   splitting the actions over two neighbouring lanes halves the accumulator
//   registers, which doubles the waves a SIMD can hold.  The two halves merge
//   their best and second-best Q with one lane shuffle (lower actions win ties).
// Weights: k = 0 takes P(D <= X_1), 0 < k < N takes P(X_1 + k) (a shift register
//   over X_1 needs one new table value per step), k = N takes P(D >= X_1 + N);
//   the tables are zero (one for the CDF) past d_max, so clipping needs no test.
// EXTRACT: write policy and Q gap instead of V (FP64 only).
template <typename VT, bool KAHAN, int RMAX, bool EXTRACT>
__global__ __launch_bounds__(512) void backup_a_kernel(ADev p) {
    extern __shared__ __align__(16) unsigned char smem[];
    Ctl* ctl = p.ctl;
    if (!EXTRACT && ctl->stop) return;
    constexpr int J = 4;
    constexpr int RH = RMAX / 2;
    constexpr int W = VecLoad<VT>::W;
    using VV = typename VecLoad<VT>::V;
    using AW = typename Acc<VT, KAHAN>::W;
    static_assert(RH % W == 0, "half row must be a whole number of vectors");

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
    // one lane per path point: its block offset once, then every action's value
    for (int j = tid; j < lp; j += bs) {
        const VT* src = vin + hbase + path_offset(j, Y, m, p.pow_y);
        VV* dst = reinterpret_cast<VV*>(S + j * RMAX);
#pragma unroll
        for (int q = 0; q < RMAX / W; ++q) {
            VT v[W];
#pragma unroll
            for (int e = 0; e < W; ++e) {
                const int a = q * W + e;
                v[e] = a < R ? src[(int64_t)a * p.stride_a] : VT(0);
            }
            dst[q] = make_vec<VT>(v);
        }
    }
    __syncthreads();

    const int G = (R + J - 1) / J;
    const int ns_tile = p.r2 * R;
    const int lanes = p.r2 * G * 2;
    const bool active = tid < lanes;
    const int half = tid & 1;
    const int cell = tid >> 1;
    const int X2 = active ? cell / G : 0;
    const int x1_0 = active ? (cell - X2 * G) * J : 0;
    const int a0 = half * RH;
    Acc<VT, KAHAN> acc[J][RH];
    if (active) {
        const int N = b + X2;
        const VT* Sh = S + a0;
        auto row_fma = [&](int pos, const AW* w) {
            const VV* row = reinterpret_cast<const VV*>(Sh + pos * RMAX);
#pragma unroll
            for (int q = 0; q < RH / W; ++q) {
                const VV u = row[q];
#pragma unroll
                for (int e = 0; e < W; ++e) {
                    const VT ue = lane_of<VT, W>(u, e);
#pragma unroll
                    for (int i = 0; i < J; ++i) acc[i][q * W + e].add(w[i], ue);
                }
            }
        };
        AW w[J];
        if (N == 0) {
#pragma unroll
            for (int i = 0; i < J; ++i) w[i] = (AW)1.0;
            row_fma(0, w);
        } else {
            const int kmax = max(0, min(N, p.dmax - x1_0));
#pragma unroll
            for (int i = 0; i < J; ++i) w[i] = (AW)sF[min(x1_0 + i, p.dmax)];
            row_fma(N, w);
            const int kend = min(N - 1, kmax);
#pragma unroll
            for (int i = 0; i < J; ++i) w[i] = (AW)sP[x1_0 + i + 1];
            for (int k = 1; k <= kend; ++k) {
                row_fma(N - k, w);
#pragma unroll
                for (int i = 0; i < J - 1; ++i) w[i] = w[i + 1];
                w[J - 1] = (AW)sP[x1_0 + J + k];
            }
            if (N <= kmax) {
#pragma unroll
                for (int i = 0; i < J; ++i) w[i] = (AW)sG[x1_0 + i + N];
                row_fma(0, w);
            }
        }
    }
    const double mu = (!EXTRACT && sizeof(VT) == 4) ? ctl->mu : 0.0;
    double dmx = -DBL_MAX, dmn = DBL_MAX, vmx = -DBL_MAX, vmn = DBL_MAX;
    double ca[RH];  // -c_var * a for this lane's actions (-inf past the last action)
#pragma unroll
    for (int e = 0; e < RH; ++e) ca[e] = a0 + e < R ? -p.cvar * (a0 + e) : -DBL_MAX;
#pragma unroll
    for (int i = 0; i < J; ++i) {
        const int X1 = x1_0 + i;
        if (EXTRACT) {
            double best = -DBL_MAX, second = -DBL_MAX;
            int arg = 0;
#pragma unroll
            for (int e = 0; e < RH; ++e) {
                if (a0 + e < R) {
                    const double q = fma(p.gamma, acc[i][e].value(), ca[e]);
                    if (q > best) {
                        second = best;
                        best = q;
                        arg = a0 + e;
                    } else if (q > second) {
                        second = q;
                    }
                }
            }
            // merge with the other half (partner lane tid ^ 1); every lane takes part
            const double ob = __shfl_xor(best, 1, 64);
            const double os = __shfl_xor(second, 1, 64);
            const int oa = __shfl_xor(arg, 1, 64);
            const double lo_b = half ? ob : best, hi_b = half ? best : ob;
            const int lo_a = half ? oa : arg, hi_a = half ? arg : oa;
            const double B = hi_b > lo_b ? hi_b : lo_b;
            const int A = hi_b > lo_b ? hi_a : lo_a;
            const double S2 = fmax(fmin(best, ob), fmax(second, os));
            if (!active || half || X1 >= R) continue;
            const int64_t s_idx = (int64_t)tile * ns_tile + X2 * R + X1;
            p.pi[s_idx] = A;
            p.gap[s_idx] = R > 1 ? B - S2 : INFINITY;
        } else {
            // a sweep needs only the max
            double best = -DBL_MAX;
#pragma unroll
            for (int e = 0; e < RH; ++e) best = fmax(best, fma(p.gamma, acc[i][e].value(), ca[e]));
            best = fmax(best, __shfl_xor(best, 1, 64));
            if (!active || half || X1 >= R) continue;
            const int64_t s_idx = (int64_t)tile * ns_tile + X2 * R + X1;
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
    span_update(ctl, a0, a1, a2, a3, fp32, fixed, gamma);
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
    constexpr int J = 4;  // states per lane (two lanes per group of states)
    const int lp_max = (p.m >= 2 ? (p.m - 2) * (p.R - 1) : 0) + p.r2;
    size_t bytes = sizeof(VT) * (size_t)lp_max * RMAX;
    bytes += sizeof(double) * (3 * (size_t)p.tab + 64);
    if (bytes > 65536) return hipErrorInvalidConfiguration;  // beyond the default LDS limit
    if (p.tab < p.R + J + lp_max || p.tab < p.dmax + 2 + J) return hipErrorInvalidValue;
    const int lanes = 2 * p.r2 * ((p.R + J - 1) / J);
    const int threads = ((lanes + 63) / 64) * 64;
    if (threads > 512) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((backup_a_kernel<VT, KAHAN, RMAX, EXTRACT>), dim3(p.tiles),
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
