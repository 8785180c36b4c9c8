// Scenario B as the paper runs it (Scenario B description, Appendix B): two
// products a and b, lead time 1, outcome = units issued (h_a, h_b), FIFO issuing,
// product b's unmet customers accept product a with probability rho.
//
// Follows the deterministic-transition update (Methods, "Value iteration").  The
// next state is (A^a, g_a(x_a, h_a), A^b, g_b(x_b, h_b)): each product ages on its
// own, and the outcome probability splits into
//   P(h_a, h_b) = [h_b < I_b] P(D_b = h_b) PA(h_a | I_a) + [h_b = I_b] J(h_a | I_a, I_b),
// where h_b = I_b leaves no stock of b (g_b = 0).  So, exactly,
//   Q(s, A) = -C_v.A + Rev(I_a, I_b) + gamma [ sum_{h_a} PA(h_a | I_a) W(A, x_b, g_a(h_a))
//                                            + Y(A, I_b, x_a) ]
//   W(A, x_b, g) = sum_{h_b < I_b} P(D_b = h_b) V(A^a, g, A^b, g_b(x_b, h_b))
//   Y(A, I_b, x_a) = sum_{h_a} J(h_a | I_a, I_b) V(A^a, g_a(x_a, h_a), A^b, 0).
// Demand up to X_1 leaves the older digits in place, and each further unit removes
// one from X_2, then X_3, ...: the aged index g walks down a path whose first point
// is x / R (the digits above X_1) and whose steps subtract R^j for the lowest digit
// j still holding stock.  The first point carries the cumulative weight of every
// outcome that ends there.  Three kernels per sweep: W, Y, then the final sum with
// the max over the joint order (ties to the lowest index) and the span partials.
#include <hip/hip_runtime.h>

#include <cfloat>

#include "device_common.h"
#include "pvi_internal.h"

namespace pvi {

namespace {

constexpr int kMaxM = PVI_MAX_LIFE;
constexpr int kCB = 16;  // orders of b per LDS chunk in the final stage (at most)

struct Digits {
    int d[kMaxM];  // d[0] = X_1 (least significant), d[k] = X_{k+1}
    int sum;
};

__device__ __forceinline__ Digits digits_of(int x, int R, int m) {
    Digits g;
    g.sum = 0;
#pragma unroll
    for (int k = 0; k < kMaxM; ++k) {
        g.d[k] = 0;
        if (k < m) {
            g.d[k] = x % R;
            x /= R;
            g.sum += g.d[k];
        }
    }
    return g;
}

// One step down the FIFO path: remove a unit from the lowest aged digit with stock.
struct PathWalk {
    int j, rem, pw;
};

__device__ __forceinline__ int step(PathWalk& w, const Digits& g, int R) {
    // callers take at most as many steps as there are units above X_1, so a digit
    // with stock is always found; the bound on j only guards the loop
    while (w.rem == 0 && w.j < kMaxM - 1) {
        ++w.j;
        w.pw *= R;
#pragma unroll
        for (int k = 1; k < kMaxM; ++k)
            if (k == w.j) w.rem = g.d[k];
    }
    --w.rem;
    return w.pw;
}

}  // namespace

// W(A, x_b, g) for one (A^a, A^b) and a block of gw values of g: the slabs
// V(A^a, g, A^b, .) sit in LDS; each output walks the path of x_b.
template <typename VT>
__global__ __launch_bounds__(256) void b1_stage_w_kernel(B1Dev p) {
    extern __shared__ __align__(16) unsigned char smem[];
    if (!p.extract && p.ctl->stop) return;
    const int ab_aa = blockIdx.y, aa = ab_aa / p.Rb, ab = ab_aa - aa * p.Rb;
    const int ga0 = blockIdx.x * p.gw, gw = min(p.gw, p.na1 - ga0);
    double* slab = reinterpret_cast<double*>(smem);  // [gw][nb1]
    const VT* V = reinterpret_cast<const VT*>(p.v_in);
    for (int i = threadIdx.x; i < gw * p.nb1; i += blockDim.x) {
        const int g = i / p.nb1, b = i - g * p.nb1;
        slab[i] = (double)V[(int64_t)(aa * p.na1 + ga0 + g) * p.NB + (int64_t)ab * p.nb1 + b];
    }
    __syncthreads();
    double* W = p.w + (int64_t)ab_aa * p.NB * p.na1;
    for (int i = threadIdx.x; i < gw * p.NB; i += blockDim.x) {
        const int g = i % gw, xb = i / gw;
        const Digits dg = digits_of(xb, p.Rb, p.m);
        const double* sl = slab + g * p.nb1;
        double acc = 0.0;
        if (dg.sum > 0) {
            const int x1 = dg.d[0], K = dg.sum - x1;
            int off = xb / p.Rb;
            acc = p.fb[min(x1, dg.sum - 1)] * sl[off];
            PathWalk w{1, dg.d[1], 1};
            for (int k = 1; k < K; ++k) {  // h_b = x1 + k < I_b
                off -= step(w, dg, p.Rb);
                acc = fma(p.pb[x1 + k], sl[off], acc);
            }
        }
        W[(int64_t)xb * p.na1 + ga0 + g] = acc;
    }
}

// Y(A, I_b, x_a) for one (A^a, A^b): the slab V(A^a, ., A^b, 0) in LDS, one lane
// per x_a, every I_b.
template <typename VT>
__global__ __launch_bounds__(256) void b1_stage_y_kernel(B1Dev p) {
    extern __shared__ __align__(16) unsigned char smem[];
    if (!p.extract && p.ctl->stop) return;
    const int ab_aa = blockIdx.y, aa = ab_aa / p.Rb, ab = ab_aa - aa * p.Rb;
    double* slab = reinterpret_cast<double*>(smem);  // [na1]
    const VT* V = reinterpret_cast<const VT*>(p.v_in);
    for (int g = threadIdx.x; g < p.na1; g += blockDim.x)
        slab[g] = (double)V[(int64_t)(aa * p.na1 + g) * p.NB + (int64_t)ab * p.nb1];
    __syncthreads();
    const int xa = blockIdx.x * blockDim.x + threadIdx.x;
    if (xa >= p.NA) return;
    const Digits dg = digits_of(xa, p.Ra, p.m);
    const int Ia = dg.sum, x1 = dg.d[0], K = Ia - x1, g0 = xa / p.Ra;
    double* Y = p.y + (int64_t)ab_aa * p.HB * p.NA + xa;
    for (int Ib = 0; Ib < p.HB; ++Ib) {
        const double* J = p.j + ((size_t)Ib * p.HA + Ia) * p.HA;
        const double* JC = p.jc + ((size_t)Ib * p.HA + Ia) * p.HA;
        int off = g0;
        double acc = JC[x1] * slab[off];
        PathWalk w{1, dg.d[1], 1};
        for (int k = 1; k <= K; ++k) {
            off -= step(w, dg, p.Ra);
            acc = fma(J[x1 + k], slab[off], acc);
        }
        Y[(int64_t)Ib * p.NA] = acc;
    }
}

// Q over the joint orders and the max, one lane per x_a, one workgroup row per x_b.
// The W slice of a chunk of orders of b sits in LDS point-major ([g][order], rows
// padded to an odd number of 16-byte units so the four paths of a wavefront fall in
// different banks), so a path point feeds the chunk's accumulators from one
// contiguous run; the weights
// come from the 1-D demand tables of a in LDS: F(x_1) at the first point (all of the
// mass when no older stock is left), P(x_1 + k) inside, P(D >= I_a) at the last.
// The 16 lanes that differ only in X_1 share the path, so their LDS reads coincide.
template <typename VT, bool EXTRACT>
__global__ __launch_bounds__(256) void b1_final_kernel(B1Dev p) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[64];
    if (!EXTRACT && p.ctl->stop) return;
    double* ws = reinterpret_cast<double*>(smem);  // [na1][cbp]
    double* wp = ws + (size_t)p.na1 * p.cbp;       // [HA + 1] P(D_a = h)
    double* wf = wp + (p.HA + 1);                  // [HA + 1] P(D_a <= h)
    double* wg = wf + (p.HA + 1);                  // [HA + 1] P(D_a >= h)
    for (int i = threadIdx.x; i <= p.HA; i += blockDim.x) {
        wp[i] = p.pa1[i];
        wf[i] = p.fa[i];
        wg[i] = p.ga[i];
    }
    // one-dimensional grid, remapped so each XCD takes contiguous runs of x_b: the
    // workgroups of one x_b read the same W slice and, for equal I_b, the same Y rows,
    // which then meet in that XCD's L2
    const int gx = (p.NA + (int)blockDim.x - 1) / (int)blockDim.x;
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int xb = lid / gx, bx = lid - xb * gx;
    const int xa = bx * blockDim.x + threadIdx.x;
    const bool ok = xa < p.NA;
    const Digits da = digits_of(ok ? xa : 0, p.Ra, p.m);
    const Digits db = digits_of(xb, p.Rb, p.m);
    const int Ia = da.sum, Ib = db.sum, x1 = da.d[0], K = Ia - x1, g0 = (ok ? xa : 0) / p.Ra;
    const double rev = p.rev[(size_t)Ia * p.HB + Ib];
    double best = -DBL_MAX, second = -DBL_MAX;
    int arg = 0;
    for (int aa = 0; aa < p.Ra; ++aa) {
        for (int ab0 = 0; ab0 < p.Rb; ab0 += p.cb) {
            const int nb = min(p.cb, p.Rb - ab0);
            __syncthreads();
            for (int i = threadIdx.x; i < nb * p.na1; i += blockDim.x) {
                const int jb = i / p.na1, g = i - jb * p.na1;
                ws[g * p.cbp + jb] = p.w[((int64_t)(aa * p.Rb + ab0 + jb) * p.NB + xb) * p.na1 + g];
            }
            __syncthreads();
            if (!ok) continue;
            double acc[kCB];
            {
                const double w0 = K > 0 ? wf[x1] : 1.0;
                const double* row = ws + g0 * p.cbp;
#pragma unroll
                for (int jb = 0; jb < kCB; ++jb) acc[jb] = jb < nb ? w0 * row[jb] : 0.0;
            }
            int off = g0;
            PathWalk w{1, da.d[1], 1};
            for (int k = 1; k <= K; ++k) {
                off -= step(w, da, p.Ra);
                const double wgt = k < K ? wp[x1 + k] : wg[Ia];
                const double* row = ws + off * p.cbp;
#pragma unroll
                for (int jb = 0; jb < kCB; ++jb)
                    if (jb < nb) acc[jb] = fma(wgt, row[jb], acc[jb]);
            }
#pragma unroll
            for (int jb = 0; jb < kCB; ++jb) {
                if (jb < nb) {
                    const int ab = ab0 + jb;
                    const double yv =
                        p.y[((int64_t)(aa * p.Rb + ab) * p.HB + Ib) * p.NA + xa];
                    const double q =
                        (-p.cva * aa - p.cvb * ab + rev) + p.gamma * (acc[jb] + yv);
                    if (q > best) {
                        second = best;
                        best = q;
                        arg = aa * p.Rb + ab;
                    } else if (q > second) {
                        second = q;
                    }
                }
            }
        }
    }
    double dmx = -DBL_MAX, dmn = DBL_MAX, vmx = -DBL_MAX, vmn = DBL_MAX;
    if (ok) {
        const int64_t s = (int64_t)xa * p.NB + xb;
        if (EXTRACT) {
            p.pi[s] = arg;
            p.gap[s] = p.Ra * p.Rb > 1 ? best - second : 0.0;
        } else {
            const double mu = sizeof(VT) == 4 ? p.ctl->mu : 0.0;
            const VT o = (VT)(best - mu);
            reinterpret_cast<VT*>(p.v_out)[s] = o;
            const double out = (double)o;
            const double dv = out - (double)reinterpret_cast<const VT*>(p.v_in)[s];
            dmx = dmn = dv;
            vmx = vmn = out;
        }
    }
    if (EXTRACT) return;
    block_reduce4(dmx, dmn, vmx, vmn, red);
    if (threadIdx.x == 0) {
        double* pp = p.partials + 4 * ((size_t)xb * gx + bx);
        pp[0] = dmx;
        pp[1] = dmn;
        pp[2] = vmx;
        pp[3] = vmn;
    }
}

// V0(s) = expected one-day sales revenue of the stock in s.
__global__ __launch_bounds__(256) void b1_initial_kernel(B1Dev p, double* v) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= (int64_t)p.NA * p.NB) return;
    const int xa = (int)(s / p.NB), xb = (int)(s - (int64_t)xa * p.NB);
    v[s] = p.rev[(size_t)digits_of(xa, p.Ra, p.m).sum * p.HB + digits_of(xb, p.Rb, p.m).sum];
}

template <typename VT, bool EXTRACT>
static hipError_t launch_b1_t(const B1Dev& p, hipStream_t s) {
    if (p.m < 1 || p.m > kMaxM || p.cb < 1 || p.cb > kCB || p.cbp < p.cb || p.gw < 1)
        return hipErrorInvalidConfiguration;
    const size_t lw = sizeof(double) * (size_t)p.gw * p.nb1;
    const size_t ly = sizeof(double) * (size_t)p.na1;
    const size_t lf = sizeof(double) * ((size_t)p.cbp * p.na1 + 3 * (size_t)(p.HA + 1));
    if (lw > 65536 || ly > 65536 || lf > 65536) return hipErrorInvalidConfiguration;
    const unsigned nact = (unsigned)(p.Ra * p.Rb);
    hipLaunchKernelGGL((b1_stage_w_kernel<VT>), dim3((p.na1 + p.gw - 1) / p.gw, nact), dim3(256),
                       lw, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned gx = (unsigned)((p.NA + 255) / 256);
    hipLaunchKernelGGL((b1_stage_y_kernel<VT>), dim3(gx, nact), dim3(256), ly, s, p);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((int64_t)gx * p.NB > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((b1_final_kernel<VT, EXTRACT>), dim3(gx * (unsigned)p.NB), dim3(256), lf,
                       s, p);
    return hipGetLastError();
}

hipError_t launch_backup_b1(const B1Dev& p, int storage_fp32, int extract, hipStream_t s) {
    if (extract) return launch_b1_t<double, true>(p, s);
    if (storage_fp32) return launch_b1_t<float, false>(p, s);
    return launch_b1_t<double, false>(p, s);
}

hipError_t launch_b1_initial(const B1Dev& p, double* v, hipStream_t s) {
    const int64_t n = (int64_t)p.NA * p.NB;
    hipLaunchKernelGGL(b1_initial_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v);
    return hipGetLastError();
}

}  // namespace pvi
