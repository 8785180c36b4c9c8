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

#include <algorithm>
#include <cfloat>

#include "device_common.h"
#include "pvi_internal.h"

namespace pvi {

// Pointer into the constant address space: loads through it whose address is the
// same for every lane go through the scalar cache.
typedef const __attribute__((address_space(4))) double* ConstF64B;

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
    // one-dimensional grid, remapped so each XCD takes contiguous runs of x_b, which come
    // in order of their digit sum I_b: the workgroups of one x_b read the same W slice
    // (in that XCD's L2), and all x_b of one I_b the same slice of Y, which stays in the
    // caches while they run
    const int gx = (p.NA + (int)blockDim.x - 1) / (int)blockDim.x;
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int xbi = lid / gx, bx = lid - xbi * gx;
    const int xb = p.xb_order[xbi];  // x_b by digit sum: equal I_b run together
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
        // this workgroup's slot (xb gx + bx = lid), and neutral values past the grid
        for (int k = lid; k < p.nslots; k += gridDim.x) {
            double* pp = p.partials + 4 * (size_t)k;
            const bool mine = k == lid;
            pp[0] = mine ? dmx : -DBL_MAX;
            pp[1] = mine ? dmn : DBL_MAX;
            pp[2] = mine ? vmx : -DBL_MAX;
            pp[3] = mine ? vmn : DBL_MAX;
        }
    }
}

// The same Q and max with the lanes over b's orders (a_max of both products below 16):
// lane (path group, ab), where a path group is x_a without X_1 (all x_a = g Ra + X_1 share
// its FIFO path), keeps 16 accumulators, one per X_1.  The lane walks its path once and
// keeps the K + 1 point offsets in registers; per order of a it then reads one W value
// (its order ab) per point from LDS, instead of the 16 orders' row that each of 16 lanes
// read in b1_final_kernel, with the 16 weights P(D_a = X_1 + k), the same for the
// whole wavefront, from the scalar cache.  The points run as straight-line code up to the
// wavefront's longest path in steps of 8; points past a lane's own path add exact zeros.
// The group's 16 x 16 sums then pass through LDS (in the W slice's space) so that lane l
// holds those of X_1 = l for every ab: its Y values are then consecutive across the lanes
// and it keeps the running maximum of its own state.  Terms, their order and the
// comparisons are those of b1_final_kernel, so V is identical.  GB path groups per
// workgroup; the W slice of one order of a, [g][ab] with rows of 17 doubles, sits in LDS.
// KMAX > the longest path (m - 1)(Ra - 1).  FP64 and FP32 storage sweeps; the policy
// extraction keeps b1_final_kernel.
template <typename VT, int GB, int KMAX>
__global__ __launch_bounds__(GB * 16) void b1_final_ab_kernel(B1Dev p) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[64];
    if (p.ctl->stop) return;
    constexpr int X1 = 16, WSP = 17, TSP = 17;
    double* ws = reinterpret_cast<double*>(smem);  // [na1][WSP], then [GB][16][TSP]
    const int ngb = (p.na1 + GB - 1) / GB;         // workgroups per x_b
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int xbi = lid / ngb, bx = lid - xbi * ngb;
    const int xb = p.xb_order[xbi];  // x_b by digit sum: equal I_b run together
    const int grp = threadIdx.x >> 4, l = threadIdx.x & 15;  // l: ab, then X_1
    const int g0 = bx * GB + grp;
    const bool gok = g0 < p.na1;
    const Digits da = digits_of(gok ? g0 * p.Ra : 0, p.Ra, p.m);  // X_1 = 0: the path group
    const int K = da.sum, Ib = digits_of(xb, p.Rb, p.m).sum;
    // the path's points (LDS offsets of their W rows); past the path, the first point
    int off[KMAX];
    int offl = g0 * WSP;  // the last point, k = K
    {
        int o = g0;
        PathWalk w{1, da.d[1], 1};
        off[0] = g0 * WSP;
#pragma unroll
        for (int k = 1; k < KMAX; ++k) {
            if (k <= K) o -= step(w, da, p.Ra);
            off[k] = (k < K ? o : g0) * WSP;
            if (k == K) offl = o * WSP;
        }
    }
    // the wavefront's longest path: the straight-line points stop there
    int kw = gok ? K : 0;
    for (int o = 32; o > 0; o >>= 1) kw = max(kw, __shfl_xor(kw, o, 64));
    kw = __builtin_amdgcn_readfirstlane(kw);
    const ConstF64B fa = (ConstF64B)p.fa;
    const ConstF64B pa = (ConstF64B)p.pa1;
    const bool sok = gok && l < p.Ra;  // lane l's state x_a = g0 Ra + l exists
    const double rev = sok ? p.rev[(size_t)(l + K) * p.HB + Ib] : 0.0;
    double best = -DBL_MAX;
    for (int aa = 0; aa < p.Ra; ++aa) {
        __syncthreads();
        for (int jb = 0; jb < p.Rb; ++jb) {
            const double* src = p.w + ((int64_t)(aa * p.Rb + jb) * p.NB + xb) * p.na1;
            for (int g = threadIdx.x; g < p.na1; g += blockDim.x) ws[g * WSP + jb] = src[g];
        }
        __syncthreads();
        double acc[X1];
        if (gok && l < p.Rb) {
            const double* wl = ws + l;
            {
                // first point: P(D_a <= X_1), or all of the mass with no older stock
                const double r0 = wl[off[0]];
#pragma unroll
                for (int i = 0; i < X1; ++i) acc[i] = (K > 0 ? fa[i] : 1.0) * r0;
            }
            // inner points k = 1 .. K-1: P(D_a = X_1 + k)
#pragma unroll
            for (int c = 1; c < KMAX; c += 8) {
                if (c >= kw) break;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int k = c + u;
                    if (k < KMAX) {
                        const double r = k < K ? wl[off[k]] : 0.0;
#pragma unroll
                        for (int i = 0; i < X1; ++i) acc[i] = fma(pa[i + k], r, acc[i]);
                    }
                }
            }
            if (K > 0) {  // last point: P(D_a >= I_a)
                const double r = wl[offl];
                const double* wg = p.ga + K;
#pragma unroll
                for (int i = 0; i < X1; ++i) acc[i] = fma(wg[i], r, acc[i]);
            }
        }
        __syncthreads();  // the W slice is read: its space takes the transposes
        double* tile = ws + grp * 16 * TSP;  // [ab][X_1]
        if (gok && l < p.Rb) {
#pragma unroll
            for (int i = 0; i < X1; ++i) tile[l * TSP + i] = acc[i];
        }
        __syncthreads();
        if (sok) {
            const double* yrow = p.y + ((int64_t)(aa * p.Rb) * p.HB + Ib) * p.NA +
                                 (int64_t)g0 * p.Ra + l;
            const int64_t ystride = (int64_t)p.HB * p.NA;  // next order of b
            for (int ab = 0; ab < p.Rb; ++ab) {
                const double yv = yrow[ab * ystride];
                const double q =
                    (-p.cva * aa - p.cvb * ab + rev) + p.gamma * (tile[ab * TSP + l] + yv);
                if (q > best) best = q;
            }
        }
    }
    double dmx = -DBL_MAX, dmn = DBL_MAX, vmx = -DBL_MAX, vmn = DBL_MAX;
    if (sok) {
        const int64_t s = ((int64_t)g0 * p.Ra + l) * p.NB + xb;
        const double mu = sizeof(VT) == 4 ? p.ctl->mu : 0.0;
        const VT o = (VT)(best - mu);
        reinterpret_cast<VT*>(p.v_out)[s] = o;
        const double out = (double)o;
        const double dv = out - (double)reinterpret_cast<const VT*>(p.v_in)[s];
        dmx = dmn = dv;
        vmx = vmn = out;
    }
    block_reduce4(dmx, dmn, vmx, vmn, red);
    if (threadIdx.x == 0) {
        // this workgroup's slot, and neutral values in the slots past the grid
        for (int k = lid; k < p.nslots; k += gridDim.x) {
            double* pp = p.partials + 4 * (size_t)k;
            const bool mine = k == lid;
            pp[0] = mine ? dmx : -DBL_MAX;
            pp[1] = mine ? dmn : DBL_MAX;
            pp[2] = mine ? vmx : -DBL_MAX;
            pp[3] = mine ? vmn : DBL_MAX;
        }
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
    if ((int64_t)gx * p.NB > 0x7fffffff || (int64_t)gx * p.NB > p.nslots)
        return hipErrorInvalidConfiguration;
    constexpr int GB = 16;  // path groups per workgroup of the lanes-over-orders kernel
    // LDS: the W slice of one order of a, which then holds the GB 16 x 17 transposes
    const size_t lab = sizeof(double) * (size_t)std::max(p.na1, GB * 16) * 17;
    const int64_t nab = (int64_t)((p.na1 + GB - 1) / GB) * p.NB;
    // the lanes-over-orders kernel where it was measured faster: 16 orders of each
    // product (fewer leave lanes idle in both 16-wide dimensions)
    const int kpath = (p.m - 1) * (p.Ra - 1);  // longest path: K points after the first
    if (!EXTRACT && p.lanes_ab && p.Ra == 16 && p.Rb == 16 && kpath < 32 && lab <= 65536 &&
        nab <= p.nslots) {
        if (kpath < 16)
            hipLaunchKernelGGL((b1_final_ab_kernel<VT, GB, 16>), dim3((unsigned)nab),
                               dim3(GB * 16), lab, s, p);
        else
            hipLaunchKernelGGL((b1_final_ab_kernel<VT, GB, 32>), dim3((unsigned)nab),
                               dim3(GB * 16), lab, s, p);
        return hipGetLastError();
    }
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
