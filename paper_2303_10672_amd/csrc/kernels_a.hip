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

// Value staged for the padding actions R <= a < RMAX: so negative that their Q
// never wins the max, small enough that weighted sums of it (total weight <= 1)
// stay finite.  With it the action loops need no bound check.
template <typename VT>
__device__ constexpr VT kPadValue = VT(-1e30);
template <>
__device__ constexpr double kPadValue<double> = -1e300;

// One wavefront per tile; VT: storage type of V (float = centred FP32, double = FP64);
// KAHAN: FP32 compensated accumulation (only with VT = float), else FP64.
// EXTRACT: write policy and Q gap instead of V (FP64 only).
//
// For a state (X_2, X_1) of the tile put N = b + X_2 (its path length, b the sum
// of the tile's fixed digits) and u = X_1 + N.  For N >= 1,
//   E = F(X_1) S[N] + C(u, N) + G(u) S[0],   C(u, N) = sum_{j=1}^{N-1} P(u - j) S[j],
// with F = P(D <= .), G = P(D >= .) and S the staged path list.  For a fixed u,
// C(u, N) is a running sum over the path points, so lane u accumulates it once for
// every action (in registers) while N walks up the list, and emits the states of
// its diagonal (X_1 = u - N in [0, R)) as N passes them.  The single-point state
// (N = 0, only when b = 0) takes S[0] for every demand.  All actions live in one
// lane, so the max needs no exchange.
template <typename VT, bool KAHAN, int RMAX, bool EXTRACT>
__global__ __launch_bounds__(64) void backup_a_kernel(ADev p) {
    extern __shared__ __align__(16) unsigned char smem[];
    Ctl* ctl = p.ctl;
    if (!EXTRACT && ctl->stop) return;
    constexpr int W = VecLoad<VT>::W;
    using VV = typename VecLoad<VT>::V;
    using AW = typename Acc<VT, KAHAN>::W;

    const int R = p.R, m = p.m, lane = threadIdx.x;
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

    // weights staged premultiplied by gamma, so that sums of weighted values are
    // already discounted
    const double g = p.gamma;
    for (int i = lane; i < p.tab; i += 64) {
        sP[i] = g * p.pmf[i];
        sF[i] = g * p.cdf[i];
        sG[i] = g * p.tail[i];
    }
    const VT* vin = reinterpret_cast<const VT*>(p.v_in);
    const int64_t hbase = (int64_t)h * p.stride_h;
    // one lane per path point: its block offset once, then every action's value
    for (int j = lane; j < lp; j += 64) {
        const VT* src = vin + hbase + path_offset(j, Y, m, p.pow_y);
        VV* dst = reinterpret_cast<VV*>(S + j * RMAX);
#pragma unroll
        for (int q = 0; q < RMAX / W; ++q) {
            VT v[W];
#pragma unroll
            for (int e = 0; e < W; ++e) {
                const int a = q * W + e;
                v[e] = a < R ? src[(int64_t)a * p.stride_a] : kPadValue<VT>;
            }
            dst[q] = make_vec<VT>(v);
        }
    }
    __syncthreads();

    const int ns_tile = p.r2 * R;
    const double mu = (!EXTRACT && sizeof(VT) == 4) ? ctl->mu : 0.0;
    double dmx = -DBL_MAX, dmn = DBL_MAX, vmx = -DBL_MAX, vmn = DBL_MAX;

    // Writes one state from the Q of its actions: the policy and gap, or V' and
    // the running max/min of V' - V and of V'.
    // r0n and vold are the state's reward-table entry and its current value,
    // loaded ahead of time by the caller.
    auto finish = [&](int X2, int X1, double best, double second, int arg, double r0n,
                      double vold) {
        const int64_t s_idx = (int64_t)tile * ns_tile + X2 * R + X1;
        if (EXTRACT) {
            p.pi[s_idx] = arg;
            p.gap[s_idx] = R > 1 ? best - second : INFINITY;
        } else {
            const VT o = (VT)(r0n - mu + best);
            reinterpret_cast<VT*>(p.v_out)[s_idx] = o;
            const double out = (double)o, dv = out - vold;
            dmx = fmax(dmx, dv);
            dmn = fmin(dmn, dv);
            vmx = fmax(vmx, out);
            vmn = fmin(vmn, out);
        }
    };
    auto take = [&](double qv, int a, double& best, double& second, int& arg) {
        if (EXTRACT) {
            if (qv > best) {
                second = best;
                best = qv;
                arg = a;
            } else if (qv > second) {
                second = qv;
            }
        } else {
            best = fmax(best, qv);
        }
    };

    // N = 0 (only when b = 0): nothing left to deplete, every demand lands on S[0]
    if (b == 0 && lane < R) {
        double r0n = 0.0, vold = 0.0;
        if (!EXTRACT) {
            r0n = p.r0[lane * p.xt + lane];
            vold = (double)vin[(int64_t)tile * ns_tile + lane];
        }
        const VV* rz = reinterpret_cast<const VV*>(S);
        double best = -DBL_MAX, second = -DBL_MAX;
        int arg = 0;
#pragma unroll
        for (int q = 0; q < RMAX / W; ++q) {
            const VV s0 = rz[q];
#pragma unroll
            for (int e = 0; e < W; ++e) {
                const int a = q * W + e;
                take(fma(g, (double)lane_of<VT, W>(s0, e), -p.cvar * a), a, best, second, arg);
            }
        }
        finish(0, lane, best, second, arg, r0n, vold);
    }
    const int nmin = b > 1 ? b : 1, nmax = b + p.r2 - 1;
    const int u = nmin + lane;  // this lane's diagonal
    const bool live = u <= nmax + R - 1;
    // The accumulator starts from the j = 0 term G(u) S[0] (and, for FP64
    // accumulation, the order cost), so a state needs only F(X_1) S[N] on top.
    Acc<VT, KAHAN> acc[RMAX];
    {
        const AW g0 = (AW)(live ? sG[u] : 0.0);
        const VV* rz = reinterpret_cast<const VV*>(S);
#pragma unroll
        for (int q = 0; q < RMAX / W; ++q) {
            const VV s0 = rz[q];
#pragma unroll
            for (int e = 0; e < W; ++e) {
                const int a = q * W + e;
                if constexpr (KAHAN)
                    acc[a].add(g0, lane_of<VT, W>(s0, e));
                else
                    acc[a].s = fma((double)g0, (double)lane_of<VT, W>(s0, e), -p.cvar * a);
            }
        }
    }
    // The lane's state at step N is X_1 = u - N, X_2 = N - b; its reward-table
    // entry and old value are fetched one step ahead so the loads overlap the
    // arithmetic.
    auto emits = [&](int N) {
        const int X1 = u - N;
        return N >= nmin && N <= nmax && live && X1 >= 0 && X1 < R;
    };
    double r0n = 0.0, vold = 0.0;
    auto prefetch = [&](int N) {
        if (!EXTRACT && emits(N)) {
            const int X1 = u - N, X2 = N - b;
            r0n = p.r0[X1 * p.xt + X1 + X2 + b];
            vold = (double)vin[(int64_t)tile * ns_tile + X2 * R + X1];
        }
    };
    prefetch(1);
    for (int N = 1; N <= nmax; ++N) {
        // one read of path point N serves the states emitted here and the running sum
        const VV* rN = reinterpret_cast<const VV*>(S + N * RMAX);
        VV sn[RMAX / W];
#pragma unroll
        for (int q = 0; q < RMAX / W; ++q) sn[q] = rN[q];
        // both weights read up front (clamped indices, always in the table) so the
        // reads overlap the arithmetic
        const int di = u - N;  // = X_1 of the state emitted here
        const double fwr = sF[min(max(di, 0), p.dmax)];
        const double pwr = sP[min(max(di, 0), p.tab - 1)];
        const double r0c = r0n, voldc = vold;
        prefetch(N + 1);
        if (emits(N)) {
            // Q_a = gamma (F(X_1) S[N][a] + C(u, N) + G(u) S[0][a]) - c_var a
            double best = -DBL_MAX, second = -DBL_MAX;
            int arg = 0;
            if constexpr (EXTRACT) {
#pragma unroll
                for (int q = 0; q < RMAX / W; ++q) {
#pragma unroll
                    for (int e = 0; e < W; ++e) {
                        const int a = q * W + e;
                        const double sv = (double)lane_of<VT, W>(sn[q], e);
                        take(fma(fwr, sv, acc[a].value()), a, best, second, arg);
                    }
                }
            } else {
                // four independent max chains, merged at the end
                double bq[4] = {-DBL_MAX, -DBL_MAX, -DBL_MAX, -DBL_MAX};
#pragma unroll
                for (int q = 0; q < RMAX / W; ++q) {
#pragma unroll
                    for (int e = 0; e < W; ++e) {
                        const int a = q * W + e;
                        const double sv = (double)lane_of<VT, W>(sn[q], e);
                        const double qv = KAHAN ? fma(fwr, sv, acc[a].value()) - p.cvar * a
                                                : fma(fwr, sv, acc[a].value());
                        bq[a & 3] = fmax(bq[a & 3], qv);
                    }
                }
                best = fmax(fmax(bq[0], bq[1]), fmax(bq[2], bq[3]));
            }
            finish(N - b, di, best, second, arg, r0c, voldc);
        }
        if (N == nmax) break;
        // add path point j = N with weight P(u - N) (zero below 1; the table is
        // zero past d_max); lanes past the last diagonal add nothing
        const AW w = (AW)(live && di >= 1 ? pwr : 0.0);
#pragma unroll
        for (int q = 0; q < RMAX / W; ++q) {
#pragma unroll
            for (int e = 0; e < W; ++e) acc[q * W + e].add(w, lane_of<VT, W>(sn[q], e));
        }
    }
    if (EXTRACT) return;
    dmx = wave_max(dmx);
    dmn = wave_min(dmn);
    vmx = wave_max(vmx);
    vmn = wave_min(vmn);
    if (lane == 0) {
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
    const int lp_max = (p.m >= 2 ? (p.m - 2) * (p.R - 1) : 0) + p.r2;
    size_t bytes = sizeof(VT) * (size_t)lp_max * RMAX;
    bytes += sizeof(double) * 3 * (size_t)p.tab;
    if (bytes > 65536) return hipErrorInvalidConfiguration;  // beyond the default LDS limit
    // lanes cover u = N + X_1 for every emitted state: at most 2R - 1 diagonals
    if (p.r2 + p.R - 1 > 64) return hipErrorInvalidConfiguration;
    if (p.tab < p.R + lp_max + 1 || p.tab < p.dmax + 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL((backup_a_kernel<VT, KAHAN, RMAX, EXTRACT>), dim3(p.tiles), dim3(64),
                       bytes, s, p);
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
