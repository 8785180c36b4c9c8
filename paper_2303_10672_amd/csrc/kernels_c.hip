// Scenario C (weekday demand, random remaining life on arrival, capacity a_max per
// life class, L = 0) Bellman backup.
//
// Follows the deterministic-transition update (Methods, "Value iteration") with T
// from Appendix C (state-transition equation, reward equation, age-on-arrival
// distribution).  The outcome is (d, y): demand d and the split y = (y_m..y_1) of
// the order over remaining lives, with probability P(d|tau) Mult(y; a, p).
// Because P factorises and the demand acts only on the post-arrival stock
// z = (y_m, min(x_{m-1}+y_{m-1}, a_max), ..., min(x_1+y_1, a_max)), the sum is
// taken in two exact stages:
//
//  stage U   U(tau, z) = sum_d P(d|tau) [ r(z, d) + gamma V(tau+1, f(z, d)) ]
//            for every z in [0, a_max]^m.  Demand up to z_1 leaves (z_m..z_2)
//            intact; z_1 + k removes k of them oldest first, so the sum walks a
//            descending path list staged in LDS, as in scenario A.
//  stage Y   Mult(y; a, p) = Bin(y_m; a, p_m) Bin(y_{m-1}; a-y_m, q_{m-1}) ...
//            with q_j = p_j / (p_1 + ... + p_j), so the arrival sum is a chain of
//            binomial merges, one life class at a time:
//              T_2(.., x_2, x_1; r)  = sum_y Bin(y; r, q_2) U(.., c(x_2+y), c(x_1+r-y))
//              T_j(.., x_j, ..; r)   = sum_y Bin(y; r, q_j) T_{j-1}(.., c(x_j+y), ..; r-y)
//              Q(tau, x, a) = -C_f[a>0] + sum_y Bin(y; a, p_m) T_{m-1}(tau, y, x; a-y)
//            where c(.) caps at a_max and r counts units still to place.
// When the remaining-life probabilities depend on the order size (the endogenous
// case, c_1 != 0), every q_j and p_m depends on a, so the merge chain runs once per
// order a with that a's factors, over the rows y_m + r <= a only; its top level
// keeps just the row r = a - y_m that the final sum for a reads, in a table of
// its own.  T tables are laid out [tau][(y_m, r) pair][x digits] so consecutive
// lanes touch consecutive addresses.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cfloat>
#include <cmath>

#include "device_common.h"
#include "pvi_internal.h"

namespace pvi {

// Offset in a next-state block of point j of the descending path list of the
// upper digits Y[2..m-1] (see the scenario-A kernel for the construction).
__device__ __forceinline__ int c_path_offset(int j, const int* Y, int m, const int* pw) {
    int off = 0;
    for (int i = m - 1; i >= 2; --i) {
        if (j < Y[i]) return off + j * pw[i - 1];
        j -= Y[i];
        off += Y[i] * pw[i - 1];
    }
    return off + j;
}

// U[tau][z_m..z_1]: one workgroup per (tau, z_m..z_3), lanes over (z_2, 4 of z_1).
template <typename VT>
__global__ __launch_bounds__(256) void c_stage_u_kernel(CDev p) {
    extern __shared__ __align__(16) unsigned char smem[];
    if (!p.extract && p.ctl->stop) return;
    constexpr int J = 4;
    const int R = p.R, m = p.m, tid = threadIdx.x;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int tau = tile / p.nzu;
    int Y[10];
    int b = 0;
    {
        int t = tile - tau * p.nzu;
        for (int i = 2; i <= m - 1; ++i) {  // Y[i] = z_{i+1}
            Y[i] = t % R;
            t /= R;
            b += Y[i];
        }
    }
    const int lp = b + R;
    double* S = reinterpret_cast<double*>(smem);
    double* sP = S + p.lpmax;
    double* sF = sP + p.tab;
    double* sG = sF + p.tab;
    const double* gP = p.pmf + (size_t)tau * p.tab;
    const double* gF = p.cdf + (size_t)tau * p.tab;
    const double* gG = p.tail + (size_t)tau * p.tab;
    for (int i = tid; i < p.tab; i += blockDim.x) {
        sP[i] = gP[i];
        sF[i] = gF[i];
        sG[i] = gG[i];
    }
    const int taun = tau + 1 == p.P ? 0 : tau + 1;
    const VT* vblk = reinterpret_cast<const VT*>(p.v_in) + (int64_t)taun * p.nblk;
    for (int j = tid; j < lp; j += blockDim.x) S[j] = (double)vblk[c_path_offset(j, Y, m, p.pow_r)];
    __syncthreads();
    const int G = (R + J - 1) / J;
    if (tid >= R * G) return;
    const int z2 = tid / G, z1_0 = (tid - z2 * G) * J;
    const int N = b + z2;
    const int kmax = N == 0 ? 0 : max(0, min(N, p.dmax - z1_0));
    double acc[J] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k <= kmax; ++k) {
        const double u = S[N - k];
#pragma unroll
        for (int i = 0; i < J; ++i) {
            const int z1 = z1_0 + i;
            const double w = N == 0 ? (k == 0 ? 1.0 : 0.0)
                             : k == 0 ? sF[min(z1, p.dmax)]
                             : k == N ? sG[z1 + N]
                                      : sP[z1 + k];
            acc[i] = fma(w, u, acc[i]);
        }
    }
    VT* U = reinterpret_cast<VT*>(p.u);
    const int64_t base = (int64_t)tile * R * R + (int64_t)z2 * R;
    const double* r0 = p.r0 + (size_t)tau * R * p.xt;
#pragma unroll
    for (int i = 0; i < J; ++i) {
        const int z1 = z1_0 + i;
        if (z1 < R) U[base + z1] = (VT)(r0[z1 * p.xt + z1 + z2 + b] + p.gamma * acc[i]);
    }
}

// Pointer into the constant address space: loads through it whose address is the
// same for every lane go through the scalar cache.
typedef const __attribute__((address_space(4))) double* ConstF64;
typedef const __attribute__((address_space(4))) int32_t* ConstI32;

// Rows r .. nr-1 of one lane's first merge, one row per template instance: term
// (r, y) reads the slab at the lane's offsets for c(x_2 + y) and c(x_1 + r - y).
template <typename VT, int RC, int r>
__device__ __forceinline__ void c_merge2_rows(const double* slab, const int (&o2)[RC],
                                              const int (&o1)[RC], ConstF64 w, int R, int nr,
                                              int rfirst, VT* out, int64_t nblk) {
    if constexpr (r < RC) {
        if (r >= nr) return;
        if (r >= rfirst) {
            const ConstF64 wr = w + r * R;
            double acc = 0.0;
#pragma unroll
            for (int y = 0; y <= r; ++y) acc = fma(wr[y], slab[o2[y] + o1[r - y]], acc);
            out[(int64_t)r * nblk] = (VT)acc;
        }
        c_merge2_rows<VT, RC, r + 1>(slab, o2, o1, w, R, nr, rfirst, out, nblk);
    }
}

// First merge (life class 2) straight from U.  One workgroup per (tau, y_m, digits
// above 2): the R x R slab U[.., z_2, z_1] sits in LDS and each lane (x_2, x_1)
// produces T_2 for every remaining count r:
//   T_2(r) = sum_{y<=r} Bin(y; r, q_2) U(.., c(x_2 + y), c(x_1 + r - y)),
// terms added in the order y = 0, 1, .., r, both sums unrolled up to RC >= R.
template <typename VT, int RC>
__global__ __launch_bounds__(1024) void c_merge2_kernel(CDev p, const void* in_, void* out_) {
    __shared__ double slab[32 * 32];
    if (!p.extract && p.ctl->stop) return;
    const int R = p.R, tid = threadIdx.x;
    const int tym = blockIdx.y, tau = tym / R, ym = tym - tau * R;
    const int64_t hi = blockIdx.x;  // digits 3..m-1
    const int nr = min(R - ym, p.alim - ym + 1);  // r = 0 .. min(a_max, alim) - y_m
    if (nr <= 0) return;
    const VT* U = reinterpret_cast<const VT*>(in_) + ((int64_t)tau * R + ym) * p.nblk + hi * R * R;
    for (int i = tid; i < R * R; i += blockDim.x) slab[i] = (double)U[i];
    __syncthreads();
    if (tid >= R * R) return;
    const int x2 = tid / R, x1 = tid - x2 * R;
    int o2[RC], o1[RC];  // slab offsets of c(x_2 + y) rows and c(x_1 + k) columns
#pragma unroll
    for (int y = 0; y < RC; ++y) {
        o2[y] = min(x2 + y, R - 1) * R;
        o1[y] = min(x1 + y, R - 1);
    }
    const ConstF64 w = (ConstF64)(p.binq + (size_t)2 * R * R);
    VT* T = reinterpret_cast<VT*>(out_) + ((int64_t)tau * p.npair + p.pair_base[ym]) * p.nblk +
            hi * R * R + tid;
    c_merge2_rows<VT, RC, 0>(slab, o2, o1, w, R, nr, p.top_only ? nr - 1 : 0, T, p.nblk);
}

// Rows r .. nr-1 of one lane's merge output (rows below rfirst skipped), one row per
// template instance so that each row's sum has a compile-time length r + 1.
template <typename VT, int LB, int RC, int r>
__device__ __forceinline__ void c_merge_rows(const VT* slab, const int (&zoff)[RC], ConstF64 w,
                                             int R, int nr, int rfirst, VT* out,
                                             int64_t nblk) {
    if constexpr (r < RC) {
        if (r >= nr) return;
        if (r >= rfirst) {
            constexpr int RS = RC * LB;
            const ConstF64 wr = w + r * R;
            double acc = 0.0;
#pragma unroll
            for (int y = 0; y <= r; ++y)
                acc = fma(wr[y], (double)slab[(r - y) * RS + zoff[y]], acc);
            out[(int64_t)r * nblk] = (VT)acc;
        }
        c_merge_rows<VT, LB, RC, r + 1>(slab, zoff, w, R, nr, rfirst, out, nblk);
    }
}

// One row of a merge of level j >= 3 from its slab: terms y = 0, 1, .., r in order.
template <typename VT, int LB, int RC, int r>
__device__ __forceinline__ double c_merge_row(const VT* slab, const int (&zoff)[RC], ConstF64 w,
                                              int R) {
    constexpr int RS = RC * LB;
    const ConstF64 wr = w + r * R;
    double acc = 0.0;
#pragma unroll
    for (int y = 0; y <= r; ++y) acc = fma(wr[y], (double)slab[(r - y) * RS + zoff[y]], acc);
    return acc;
}

// Rows r .. nr-1 of a lane's merge output (every row), four rows per block as above.
template <typename VT, int LB, int RC, int r>
__device__ __forceinline__ void c_merge_rows4(const VT* slab, const int (&zoff)[RC], ConstF64 w,
                                              int R, int nr, VT* out, int64_t nblk) {
    if constexpr (r + 3 < RC) {
        if (r + 3 < nr) {
            const double a0 = c_merge_row<VT, LB, RC, r>(slab, zoff, w, R);
            const double a1 = c_merge_row<VT, LB, RC, r + 1>(slab, zoff, w, R);
            const double a2 = c_merge_row<VT, LB, RC, r + 2>(slab, zoff, w, R);
            const double a3 = c_merge_row<VT, LB, RC, r + 3>(slab, zoff, w, R);
            out[(int64_t)r * nblk] = (VT)a0;
            out[(int64_t)(r + 1) * nblk] = (VT)a1;
            out[(int64_t)(r + 2) * nblk] = (VT)a2;
            out[(int64_t)(r + 3) * nblk] = (VT)a3;
            c_merge_rows4<VT, LB, RC, r + 4>(slab, zoff, w, R, nr, out, nblk);
            return;
        }
    }
    if constexpr (r < RC) {
        if (r < nr) out[(int64_t)r * nblk] = (VT)c_merge_row<VT, LB, RC, r>(slab, zoff, w, R);
    }
    if constexpr (r + 1 < RC) {
        if (r + 1 < nr)
            out[(int64_t)(r + 1) * nblk] = (VT)c_merge_row<VT, LB, RC, r + 1>(slab, zoff, w, R);
    }
    if constexpr (r + 2 < RC) {
        if (r + 2 < nr)
            out[(int64_t)(r + 2) * nblk] = (VT)c_merge_row<VT, LB, RC, r + 2>(slab, zoff, w, R);
    }
}

// Merge of life class j >= 3.  One workgroup per (tau, y_m, digits above j, block of
// LB consecutive values of the digits below j); the slab in[r'][z_j][lo] for every
// remaining count r' is staged in LDS once, and each lane (x_j, lo) produces
//   T_j(r) = sum_{y<=r} Bin(y; r, q_j) T_{j-1}(.., c(x_j + y), ..; r - y)
// for every r.  Lanes with consecutive lo touch consecutive addresses; each lane
// stages one (z_j, lo) column over all r', so no index division runs per element.
// Both sums are unrolled at compile time up to RC >= R: rows of the slab are RC * LB
// apart, so term (r, y) is an LDS read at the lane's offset for c(x_j + y) plus the
// constant (r - y) RC LB, the reads of a row can all be in flight at once, and the
// binomial weights, the same for every lane, come through the scalar cache.  Terms
// are added in the order y = 0, 1, .., r.  The grid is one-dimensional and remapped
// so that each XCD takes a contiguous run of blocks: neighbouring lo-blocks share
// cache lines, which then meet in one L2.
template <typename VT, int LB, int RC>
__global__ __launch_bounds__(1024) void c_merge_kernel(CDev p, int j, const void* in_,
                                                       void* out_) {
    extern __shared__ __align__(16) unsigned char smem[];
    if (!p.extract && p.ctl->stop) return;
    constexpr int RS = RC * LB;  // slab row stride
    const int R = p.R, tid = threadIdx.x;
    VT* slab = reinterpret_cast<VT*>(smem);  // [r'][z < RC][LB]
    // block decomposition in 32 bits (the launcher checks that the counts fit)
    const int nlo = (int)p.pow_r[j - 1];  // R^(j-1) values below digit j
    const int nlob = (nlo + LB - 1) / LB;
    const int nx = (int)(p.nblk / ((int64_t)nlo * R)) * nlob;  // blocks per (tau, y_m)
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int tym = lid / nx, tau = tym / R, ym = tym - tau * R;
    const int xb = lid - tym * nx;
    const int nr = min(R - ym, p.alim - ym + 1);
    if (nr <= 0) return;
    const int hi = xb / nlob;
    const int lo0 = (xb - hi * nlob) * LB;
    const int64_t base = (int64_t)hi * nlo * R + lo0;  // digits above j, digit j = 0, lo0
    const int64_t row0 = (int64_t)tau * p.npair + p.pair_base[ym];
    const int l = tid % LB, xz = tid / LB;  // lane: lo offset, digit j value
    const bool lane_ok = xz < R && lo0 + l < nlo;
    const VT* in = reinterpret_cast<const VT*>(in_);
    if (xz < R) {
        // every row's load is issued before the first LDS write waits for one
        const VT* src = in + row0 * p.nblk + base + (int64_t)xz * nlo + l;
        const bool ok = lo0 + l < nlo;
        VT v[RC];
#pragma unroll
        for (int rr = 0; rr < RC; ++rr)
            v[rr] = ok && rr < nr ? src[(int64_t)rr * p.nblk] : VT(0);
#pragma unroll
        for (int rr = 0; rr < RC; ++rr)
            if (rr < nr) slab[rr * RS + xz * LB + l] = v[rr];
    }
    __syncthreads();
    if (!lane_ok) return;
    int zoff[RC];  // slab offset of column c(x_j + y) in row 0
#pragma unroll
    for (int y = 0; y < RC; ++y) zoff[y] = min(xz + y, R - 1) * LB + l;
    // weights Bin(y; r, q_j) at r R + y
    const ConstF64 w = (ConstF64)(p.binq + (size_t)j * R * R);
    VT* out = reinterpret_cast<VT*>(out_) + row0 * p.nblk + base + (int64_t)xz * nlo + l;
    if (p.top_only)
        c_merge_rows<VT, LB, RC, 0>(slab, zoff, w, R, nr, nr - 1, out, p.nblk);
    else
        c_merge_rows4<VT, LB, RC, 0>(slab, zoff, w, R, nr, out, p.nblk);
}

// Orders a .. R-1 of one state's final sum (m >= 3), one order per template instance so
// that its a + 1 table reads can all be in flight: Q(a) = -C_f [a > 0] +
// sum_{y<=a} Bin(y; a, p_m) T(row(y) + a - y, D), then the running best, second and
// argmax in order of a (the plain loop's order and arithmetic).
template <typename VT, int RC, int a>
__device__ __forceinline__ void c_final_orders(const VT* T, ConstF64 bm, ConstI32 pb,
                                               int64_t rowbase, int64_t nblk, int64_t D,
                                               int R, double cfixed, double& best,
                                               double& second, int& arg) {
    if constexpr (a < RC) {
        if (a >= R) return;
        const ConstF64 w = bm + a * R;
        double acc = 0.0;
#pragma unroll
        for (int y = 0; y <= a; ++y)
            acc = fma(w[y], (double)T[(rowbase + pb[y] + (a - y)) * nblk + D], acc);
        const double q = (a > 0 ? -cfixed : 0.0) + acc;
        if (q > best) {
            second = best;
            best = q;
            arg = a;
        } else if (q > second) {
            second = q;
        }
        c_final_orders<VT, RC, a + 1>(T, bm, pb, rowbase, nblk, D, R, cfixed, best, second,
                                      arg);
    }
}

// Q(tau, x, a) = -C_f [a > 0] + sum_y Bin(y; a, p_m) T_{m-1}(tau, y, x; a - y), then
// the max over a.  One lane per state.
template <typename VT, bool EXTRACT, int RC>
__global__ __launch_bounds__(256) void c_final_kernel(CDev p, const void* tin) {
    __shared__ double red[64];
    if (!EXTRACT && p.ctl->stop) return;
    const int R = p.R;
    const int tau = blockIdx.y;
    const int64_t D = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double dmx = -DBL_MAX, dmn = DBL_MAX, vmx = -DBL_MAX, vmn = DBL_MAX;
    if (D < p.nblk) {
        const VT* T = reinterpret_cast<const VT*>(tin);
        double best = -DBL_MAX, second = -DBL_MAX;
        int arg = 0;
        if (p.m == 2) {
            // no middle life classes: T_1 is U with digit 1 capped
            for (int a = 0; a < R; ++a) {
                double acc = 0.0;
                for (int y = 0; y <= a; ++y) {
                    const VT* U = T + ((int64_t)tau * R + y) * p.nblk;
                    acc = fma(p.binm[a * R + y], (double)U[min((int)D + (a - y), R - 1)], acc);
                }
                const double q = (a > 0 ? -p.cfixed : 0.0) + acc;
                if (q > best) {
                    second = best;
                    best = q;
                    arg = a;
                } else if (q > second) {
                    second = q;
                }
            }
        } else {
            c_final_orders<VT, RC, 0>(T, (ConstF64)p.binm, (ConstI32)p.pair_base,
                                      (int64_t)tau * p.npair, p.nblk, D, R, p.cfixed, best,
                                      second, arg);
        }
        const int64_t s = (int64_t)tau * p.nblk + D;
        if (EXTRACT) {
            p.pi[s] = arg;
            p.gap[s] = best - second;
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
        double* pp = p.partials + 4 * ((size_t)tau * gridDim.x + blockIdx.x);
        pp[0] = dmx;
        pp[1] = dmn;
        pp[2] = vmx;
        pp[3] = vmn;
    }
}

// One row of the first merge from a U plane: terms y = 0, 1, .., r in order.
template <typename VT, int RC, int r>
__device__ __forceinline__ double c23_first_row(const VT* plane, const int (&o2)[RC],
                                                const int (&o1)[RC], ConstF64 w, int R) {
    const ConstF64 wr = w + r * R;
    double acc = 0.0;
#pragma unroll
    for (int y = 0; y <= r; ++y) acc = fma(wr[y], (double)plane[o2[y] + o1[r - y]], acc);
    return acc;
}

// Rows r .. nr-1 of the lane's first merge into its slab column (rows rs apart), four
// rows per block where all four exist, so that their independent chains of
// multiply-adds interleave; each row's own terms stay in order.
template <typename VT, int RC, int r>
__device__ __forceinline__ void c23_first_rows(const VT* plane, const int (&o2)[RC],
                                               const int (&o1)[RC], ConstF64 w, int R, int nr,
                                               VT* col, int rs) {
    if constexpr (r + 3 < RC) {
        if (r + 3 < nr) {
            const double a0 = c23_first_row<VT, RC, r>(plane, o2, o1, w, R);
            const double a1 = c23_first_row<VT, RC, r + 1>(plane, o2, o1, w, R);
            const double a2 = c23_first_row<VT, RC, r + 2>(plane, o2, o1, w, R);
            const double a3 = c23_first_row<VT, RC, r + 3>(plane, o2, o1, w, R);
            col[r * rs] = (VT)a0;
            col[(r + 1) * rs] = (VT)a1;
            col[(r + 2) * rs] = (VT)a2;
            col[(r + 3) * rs] = (VT)a3;
            c23_first_rows<VT, RC, r + 4>(plane, o2, o1, w, R, nr, col, rs);
            return;
        }
    }
    if constexpr (r < RC) {
        if (r < nr) col[r * rs] = (VT)c23_first_row<VT, RC, r>(plane, o2, o1, w, R);
    }
    if constexpr (r + 1 < RC) {
        if (r + 1 < nr) col[(r + 1) * rs] = (VT)c23_first_row<VT, RC, r + 1>(plane, o2, o1, w, R);
    }
    if constexpr (r + 2 < RC) {
        if (r + 2 < nr) col[(r + 2) * rs] = (VT)c23_first_row<VT, RC, r + 2>(plane, o2, o1, w, R);
    }
}

// Merges of life classes 2 and 3 in one kernel (m >= 5): T_3 straight from U, so T_2 is
// never stored.  One workgroup per (y_m, tau, digits above 3), longest rows (small y_m)
// first; it stages the whole cube U(tau, y_m, .., z_3, z_2, z_1) (R^3 values) in LDS once
// and walks the blocks of LB consecutive values lo = (x_2, x_1).  Per block, lane
// (z_3, lo) first forms its slab column
//   T_2(z_3, lo; r') = sum_{y<=r'} Bin(y; r', q_2) U(z_3, c(x_2 + y), c(x_1 + r' - y))
// for every r' (the first merge kernel's terms and order, rounded to the table type),
// then, as lane (x_3, lo), the level-3 merge of the merge kernel from that slab, written
// to T_3.  The cube is read from HBM once per sweep; each term is one LDS read.
template <typename VT, int LB, int RC>
__global__ __launch_bounds__(kCFusedThreads) void c_merge23_kernel(CDev p, const void* u_,
                                                                   void* out_) {
    extern __shared__ __align__(16) unsigned char smem[];
    if (!p.extract && p.ctl->stop) return;
    constexpr int RS = RC * LB;  // slab row stride
    const int R = p.R, tid = threadIdx.x;
    const int RR = R * R, R3 = RR * R;
    VT* cube = reinterpret_cast<VT*>(smem);  // U[z_3][z_2][z_1]
    VT* slab = cube + R3;                    // T_2[r'][z_3 < RC][LB]
    const int nhi = (int)(p.nblk / R3);      // values of the digits above 3
    int b = blockIdx.x;
    const int ym = b / (p.P * nhi);
    b -= ym * p.P * nhi;
    const int tau = b / nhi, hi = b - tau * nhi;
    const int nr = min(R - ym, p.alim - ym + 1);
    if (nr <= 0) return;
    {
        const VT* U = reinterpret_cast<const VT*>(u_) + ((int64_t)tau * R + ym) * p.nblk +
                      (int64_t)hi * R3;
        for (int i = tid; i < R3; i += blockDim.x) cube[i] = U[i];
    }
    const int l = tid % LB, xz = tid / LB;  // lane: lo offset, digit 3 (z_3, then x_3)
    int zoff[RC];                           // slab offset of column c(x_3 + y) in row 0
#pragma unroll
    for (int y = 0; y < RC; ++y) zoff[y] = min(xz + y, R - 1) * LB + l;
    const ConstF64 w2 = (ConstF64)(p.binq + (size_t)2 * R * R);
    const ConstF64 w3 = (ConstF64)(p.binq + (size_t)3 * R * R);
    VT* T = reinterpret_cast<VT*>(out_) +
            ((int64_t)tau * p.npair + p.pair_base[ym]) * p.nblk + (int64_t)hi * R3 +
            (int64_t)xz * RR + l;
    const int nlob = (RR + LB - 1) / LB;
    __syncthreads();
    for (int blk = 0; blk < nlob; ++blk) {
        const int lo = blk * LB + l;
        const bool ok = xz < R && lo < RR;
        if (ok) {
            const int x2 = lo / R, x1 = lo - x2 * R;
            int o2[RC], o1[RC];  // plane offsets of c(x_2 + y) rows and c(x_1 + k) columns
#pragma unroll
            for (int y = 0; y < RC; ++y) {
                o2[y] = min(x2 + y, R - 1) * R;
                o1[y] = min(x1 + y, R - 1);
            }
            c23_first_rows<VT, RC, 0>(cube + xz * RR, o2, o1, w2, R, nr, slab + xz * LB + l,
                                      RS);
        }
        __syncthreads();
        if (ok) c_merge_rows4<VT, LB, RC, 0>(slab, zoff, w3, R, nr, T + blk * LB, p.nblk);
        __syncthreads();
    }
}

// Rows r .. nr-1 of the top merge for one y_m, each folded into the final sums at once:
// T(r) = sum_{y<=r} Bin(y; r, q_{m-1}) slab(r - y, c(x_{m-1} + y)) (the merge kernel's
// terms and order, rounded to the table type as a stored table would be), then
// B[r] += Bin(y_m; y_m + r, p_m) T(r), B[r] being the running final sum of order y_m + r.
// A compiler barrier after each row keeps the reads of later rows from being hoisted
// above it (the rows' inputs would otherwise all be live at once and spill).
template <typename VT, int LB, int RC, int r>
__device__ __forceinline__ void c_top_rows(const VT* slab, const int (&zoff)[RC], ConstF64 w,
                                           ConstF64 bm, int R, int ym, int nr,
                                           double (&B)[RC]) {
    if constexpr (r < RC) {
        if (r < nr) {
            const double t = c_merge_row<VT, LB, RC, r>(slab, zoff, w, R);
            B[r] = fma(bm[(ym + r) * R + ym], (double)(VT)t, B[r]);
        }
        asm volatile("" ::: "memory");
        c_top_rows<VT, LB, RC, r + 1>(slab, zoff, w, bm, R, ym, nr, B);
    }
}

// Top merge (life class m-1, m >= 4, order-independent life) fused with the final sum
// and the max over orders, so the top table is never written or read back:
//   Q(tau, x, a) = -C_f [a > 0] + sum_{y_m<=a} Bin(y_m; a, p_m) T_{m-1}(tau, y_m, x; a - y_m).
// One workgroup per (tau, block of LB consecutive values of the digits below m-1); lanes
// (x_{m-1}, lo) as in the merge kernel, one state each.  The loop runs over y_m; for each
// it stages the slab T_{m-2}(tau, y_m, z, lo; r') (r' < R - y_m) in LDS and adds every
// row's merge into B (other workgroups on the CU load while this one computes).  Order
// a = y_m is then complete (its terms arrive in the order y_m = 0, 1, .., a, as in the
// final kernel), so the running best, second and argmax follow the order of a, and B
// shifts down by one.  Partial slot of a workgroup: its block id; slots past the grid
// (the count is sized for the narrowest block) get neutral values.
template <typename VT, int LB, int RC>
__global__ __launch_bounds__(kCFusedThreads) void c_top_final_kernel(CDev p, const void* in_,
                                                                  int nslots) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[64];
    if (!p.extract && p.ctl->stop) return;
    constexpr int RS = RC * LB;
    const int R = p.R, tid = threadIdx.x, j = p.m - 1;
    VT* slab = reinterpret_cast<VT*>(smem);  // [r'][z < RC][LB]
    const int nlo = (int)p.pow_r[j - 1];     // R^(m-2): the digits below m-1
    const int nlob = (nlo + LB - 1) / LB;
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int tau = lid / nlob;
    const int lo0 = (lid - tau * nlob) * LB;
    const int l = tid % LB, xz = tid / LB;  // lane: lo offset, digit m-1
    const bool lane_ok = xz < R && lo0 + l < nlo;
    const int64_t D = (int64_t)xz * nlo + lo0 + l;  // the lane's state within weekday tau
    const int64_t trow = (int64_t)tau * p.npair;
    const VT* in = reinterpret_cast<const VT*>(in_);
    const ConstI32 pb = (ConstI32)p.pair_base;
    int zoff[RC];  // slab offset of column c(x_{m-1} + y) in row 0
#pragma unroll
    for (int y = 0; y < RC; ++y) zoff[y] = min(xz + y, R - 1) * LB + l;
    const ConstF64 w = (ConstF64)(p.binq + (size_t)j * R * R);
    const ConstF64 bm = (ConstF64)p.binm;
    double B[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) B[r] = 0.0;
    double best = -DBL_MAX, second = -DBL_MAX;
    int arg = 0;
    for (int ym = 0; ym < R; ++ym) {
        const int nr = R - ym;
        if (ym > 0) __syncthreads();  // the previous y_m's rows are read
        if (lane_ok) {
            // every row's load is issued before the first LDS write waits for one
            const VT* src = in + (trow + pb[ym]) * p.nblk + D;
            VT v[RC];
#pragma unroll
            for (int rr = 0; rr < RC; ++rr) v[rr] = rr < nr ? src[(int64_t)rr * p.nblk] : VT(0);
#pragma unroll
            for (int rr = 0; rr < RC; ++rr)
                if (rr < nr) slab[rr * RS + xz * LB + l] = v[rr];
        }
        __syncthreads();
        if (lane_ok) {
            // the merge weights do not change with y_m; an opaque copy of their address
            // keeps the compiler from hoisting all of them out of the loop into registers
            ConstF64 wl = w;
            asm volatile("" : "+s"(wl));
            c_top_rows<VT, LB, RC, 0>(slab, zoff, wl, bm, R, ym, nr, B);
            const double q = (ym > 0 ? -p.cfixed : 0.0) + B[0];
            if (q > best) {
                second = best;
                best = q;
                arg = ym;
            } else if (q > second) {
                second = q;
            }
        }
#pragma unroll
        for (int r = 0; r + 1 < RC; ++r) B[r] = B[r + 1];
        B[RC - 1] = 0.0;
    }
    double dmx = -DBL_MAX, dmn = DBL_MAX, vmx = -DBL_MAX, vmn = DBL_MAX;
    if (lane_ok) {
        const int64_t s = (int64_t)tau * p.nblk + D;
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
        for (int k = lid; k < nslots; k += gridDim.x) {
            double* pp = p.partials + 4 * (size_t)k;
            const bool mine = k == lid;
            pp[0] = mine ? dmx : -DBL_MAX;
            pp[1] = mine ? dmn : DBL_MAX;
            pp[2] = mine ? vmx : -DBL_MAX;
            pp[3] = mine ? vmn : DBL_MAX;
        }
    }
}

// compile-time bound of the merge sums for R (the merge kernels' RC)
static int c_rc_for(int R) { return R <= 8 ? 8 : R <= 16 ? 16 : R <= 24 ? 24 : 32; }

// LDS of one merge workgroup: R rows of RC x lb slab values
template <typename VT>
static size_t c_lds_for(const CDev& p, int lb) {
    return sizeof(VT) * (size_t)p.R * c_rc_for(p.R) * lb;
}

template <typename VT>
static int c_default_lb(const CDev& p) {
    int lb = (int)(64 / sizeof(VT));
    while (lb > 4 && (c_lds_for<VT>(p, lb) > 32768 || p.R * lb > 1024)) lb /= 2;
    return lb;
}

template <typename VT>
static hipError_t launch_c_chain(const CDev& p, void* top, int jlast, hipStream_t s);
template <typename VT>
static hipError_t launch_merge_lb(const CDev& p, int j, const void* in, void* out, int lb,
                                  dim3 grid, int threads, size_t lds, hipStream_t s);

// block width of merge level j (tuned, else the LDS rule)
template <typename VT>
static int c_level_lb(const CDev& p, int j) {
    const int tuned = p.lb[sizeof(VT) == 4 ? 1 : 0][j];
    return tuned > 0 ? tuned : c_default_lb<VT>(p);
}

// LDS a workgroup may take on the current device (more than 64 KB on gfx950), cached
// per device.
static size_t c_device_lds() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
    int v = cache[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                hipSuccess || v <= 0)
            v = 65536;
        cache[dev].store(v, std::memory_order_relaxed);
    }
    return (size_t)v;
}

// LDS of one workgroup of the fused first two merges: the U cube and the level-3 slab
template <typename VT>
static size_t c23_lds_for(const CDev& p, int lb) {
    return sizeof(VT) * ((size_t)p.R * p.R * p.R + (size_t)p.R * c_rc_for(p.R) * lb);
}

// Whether the first two merges run fused at level-3 block width lb (m >= 5, where level 3
// is not the top level): the cube and slab must fit the device's LDS.
template <typename VT>
static bool c_use23(const CDev& p, int lb) {
    const int64_t r3 = (int64_t)p.R * p.R * p.R;
    return p.m >= 5 && p.R <= 32 && p.R * lb <= kCFusedThreads &&
           c23_lds_for<VT>(p, lb) <= c_device_lds() && p.nblk % r3 == 0 &&
           (int64_t)p.R * p.P * (p.nblk / r3) <= 0x7fffffff;
}

template <typename VT, int LB>
static hipError_t launch_merge23_rc(const CDev& p, const void* u, void* out, dim3 grid,
                                    int threads, size_t lds, hipStream_t s) {
    if (p.R <= 8)
        hipLaunchKernelGGL((c_merge23_kernel<VT, LB, 8>), grid, dim3(threads), lds, s, p, u, out);
    else if (p.R <= 16)
        hipLaunchKernelGGL((c_merge23_kernel<VT, LB, 16>), grid, dim3(threads), lds, s, p, u, out);
    else if (p.R <= 24)
        hipLaunchKernelGGL((c_merge23_kernel<VT, LB, 24>), grid, dim3(threads), lds, s, p, u, out);
    else
        hipLaunchKernelGGL((c_merge23_kernel<VT, LB, 32>), grid, dim3(threads), lds, s, p, u, out);
    return hipGetLastError();
}

// The fused first two merges at level-3 block width lb, U in `u`, T_3 into `out`.
template <typename VT>
static hipError_t launch_merge23(const CDev& p, const void* u, void* out, int lb, hipStream_t s) {
    if (!c_use23<VT>(p, lb)) return hipErrorInvalidConfiguration;
    const int64_t nhi = p.nblk / ((int64_t)p.R * p.R * p.R);
    const dim3 grid((unsigned)(p.R * p.P * nhi));
    const int threads = ((p.R * lb + 63) / 64) * 64;
    const size_t lds = c23_lds_for<VT>(p, lb);
    if (lb == 32) return launch_merge23_rc<VT, 32>(p, u, out, grid, threads, lds, s);
    if (lb == 16) return launch_merge23_rc<VT, 16>(p, u, out, grid, threads, lds, s);
    if (lb == 12) return launch_merge23_rc<VT, 12>(p, u, out, grid, threads, lds, s);
    if (lb == 8) return launch_merge23_rc<VT, 8>(p, u, out, grid, threads, lds, s);
    if (lb == 4) return launch_merge23_rc<VT, 4>(p, u, out, grid, threads, lds, s);
    return hipErrorInvalidValue;
}

template <typename VT, int LB>
static hipError_t launch_top_final_rc(const CDev& p, const void* in, int nslots, dim3 grid,
                                      int threads, size_t lds, hipStream_t s) {
    if (p.R <= 8)
        hipLaunchKernelGGL((c_top_final_kernel<VT, LB, 8>), grid, dim3(threads), lds, s, p, in, nslots);
    else if (p.R <= 16)
        hipLaunchKernelGGL((c_top_final_kernel<VT, LB, 16>), grid, dim3(threads), lds, s, p, in, nslots);
    else if (p.R <= 24)
        hipLaunchKernelGGL((c_top_final_kernel<VT, LB, 24>), grid, dim3(threads), lds, s, p, in, nslots);
    else
        hipLaunchKernelGGL((c_top_final_kernel<VT, LB, 32>), grid, dim3(threads), lds, s, p, in, nslots);
    return hipGetLastError();
}

// The fused top merge and final sum at block width lb, reading level m-2 from `in`.
template <typename VT>
static hipError_t launch_top_final(const CDev& p, const void* in, int lb, hipStream_t s) {
    const int64_t nlo = p.pow_r[p.m - 2];
    const int64_t nlob = (nlo + lb - 1) / lb;
    const int64_t nwg = nlob * p.P;
    const int64_t nslots = c_partial_slots(p.P, nlo);
    const int threads = ((p.R * lb + 63) / 64) * 64;
    const size_t lds = c_lds_for<VT>(p, lb);
    if (p.m < 4 || !p.exogenous || p.R > 32 || lds > 65536 || p.R * lb > kCFusedThreads ||
        nslots > 0x7fffffff || nwg > nslots || nlo * p.R != p.nblk)
        return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)nwg);
    const int ns = (int)nslots;
    if (lb == 32) return launch_top_final_rc<VT, 32>(p, in, ns, grid, threads, lds, s);
    if (lb == 16) return launch_top_final_rc<VT, 16>(p, in, ns, grid, threads, lds, s);
    if (lb == 12) return launch_top_final_rc<VT, 12>(p, in, ns, grid, threads, lds, s);
    if (lb == 8) return launch_top_final_rc<VT, 8>(p, in, ns, grid, threads, lds, s);
    if (lb == 4) return launch_top_final_rc<VT, 4>(p, in, ns, grid, threads, lds, s);
    return hipErrorInvalidValue;
}

template <typename VT, bool EXTRACT>
static hipError_t launch_c_t(const CDev& p, hipStream_t s) {
    const size_t ubytes = sizeof(double) * ((size_t)p.lpmax + 3 * (size_t)p.tab);
    if (ubytes > 65536) return hipErrorInvalidConfiguration;
    const int G = (p.R + 3) / 4;
    const int threads = ((p.R * G + 63) / 64) * 64;
    if (threads > 256 || p.R > 32) return hipErrorInvalidConfiguration;
    if (p.tab < p.R + 4 + p.lpmax || p.tab < p.dmax + 6) return hipErrorInvalidValue;
    hipLaunchKernelGGL((c_stage_u_kernel<VT>), dim3(p.P * p.nzu), dim3(threads), ubytes, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned gx = (unsigned)((p.nblk + 255) / 256);
    const void* tin = p.u;
    if (!EXTRACT && p.m >= 4 && p.exogenous) {
        // levels 2 .. m-2, then the top level fused with the final sum
        if ((e = launch_c_chain<VT>(p, nullptr, p.m - 2, s)) != hipSuccess) return e;
        tin = ((p.m - 2) & 1) ? p.t1 : p.t0;
        return launch_top_final<VT>(p, tin, c_level_lb<VT>(p, p.m - 1), s);
    }
    if (p.m >= 3 && p.exogenous) {
        if ((e = launch_c_chain<VT>(p, p.t1 /* level m-1 output */, p.m - 1, s)) != hipSuccess)
            return e;
        tin = ((p.m - 1) & 1) ? p.t1 : p.t0;
    } else if (p.m >= 3) {
        for (int a = 0; a < p.R; ++a) {
            CDev q = p;
            q.binq = p.binq + (size_t)a * p.m * p.R * p.R;
            q.alim = a;
            if ((e = launch_c_chain<VT>(q, p.tf, p.m - 1, s)) != hipSuccess) return e;
        }
        tin = p.tf;
    }
    const dim3 fg(gx, p.P);
    if (p.R <= 8)
        hipLaunchKernelGGL((c_final_kernel<VT, EXTRACT, 8>), fg, dim3(256), 0, s, p, tin);
    else if (p.R <= 16)
        hipLaunchKernelGGL((c_final_kernel<VT, EXTRACT, 16>), fg, dim3(256), 0, s, p, tin);
    else if (p.R <= 24)
        hipLaunchKernelGGL((c_final_kernel<VT, EXTRACT, 24>), fg, dim3(256), 0, s, p, tin);
    else
        hipLaunchKernelGGL((c_final_kernel<VT, EXTRACT, 32>), fg, dim3(256), 0, s, p, tin);
    return hipGetLastError();
}

// The merges of life classes 2 .. jlast from U.  Levels alternate between the two
// ping-pong tables (level j writes t_{j mod 2}); in the order-dependent case (alim <
// a_max possible) the top level m-1 writes only its row r = alim - y_m, into `top`.
template <typename VT>
static hipError_t launch_c_chain(const CDev& p, void* top, int jlast, hipStream_t s) {
    hipError_t e = hipSuccess;
    const void* in = p.u;
    void* bufs[2] = {p.t0, p.t1};
    for (int j = 2; j <= jlast; ++j) {
        CDev q = p;
        void* out = bufs[j & 1];
        if (!p.exogenous && j == p.m - 1) {
            q.top_only = 1;
            out = top;
        }
        if (j == 2 && jlast >= 3 && c_use23<VT>(p, c_level_lb<VT>(p, 3))) {
            // levels 2 and 3 in one kernel, T_3 into level 3's table
            out = bufs[1];
            if ((e = launch_merge23<VT>(p, in, out, c_level_lb<VT>(p, 3), s)) != hipSuccess)
                return e;
            in = out;
            ++j;
            continue;
        }
        if (j == 2) {
            const int threads = ((p.R * p.R + 63) / 64) * 64;
            const dim3 grid((unsigned)(p.nblk / (p.R * p.R)), p.P * p.R);
            if (p.R <= 8)
                hipLaunchKernelGGL((c_merge2_kernel<VT, 8>), grid, dim3(threads), 0, s, q, in, out);
            else if (p.R <= 16)
                hipLaunchKernelGGL((c_merge2_kernel<VT, 16>), grid, dim3(threads), 0, s, q, in, out);
            else if (p.R <= 24)
                hipLaunchKernelGGL((c_merge2_kernel<VT, 24>), grid, dim3(threads), 0, s, q, in, out);
            else
                hipLaunchKernelGGL((c_merge2_kernel<VT, 32>), grid, dim3(threads), 0, s, q, in, out);
        } else {
            // the tuned block width of this level, else the widest block of low digits
            // (up to 64 bytes per slab row) whose slab stays within 32 KB of LDS, so
            // several workgroups share a CU
            const int lb = c_level_lb<VT>(p, j);
            if (c_lds_for<VT>(p, lb) > 65536 || p.R * lb > 1024)
                return hipErrorInvalidConfiguration;
            auto lds_for = [&](int w) { return c_lds_for<VT>(p, w); };
            const int64_t nlo = p.pow_r[j - 1];
            const int64_t nlob = (nlo + lb - 1) / lb;
            const int64_t nhi = p.nblk / (nlo * p.R);
            const int threads = ((p.R * lb + 63) / 64) * 64;
            const int64_t nwg = nhi * nlob * p.P * p.R;
            // the kernel decomposes block ids and offsets in 32 bits
            if (nwg > 0x7fffffff || nlo * p.R > 0x7fffffff || p.R > 32)
                return hipErrorInvalidConfiguration;
            const dim3 grid((unsigned)nwg);
            const size_t lds = lds_for(lb);
            if ((e = launch_merge_lb<VT>(q, j, in, out, lb, grid, threads, lds, s)) != hipSuccess)
                return e;
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        in = out;
    }
    (void)top;
    return hipSuccess;
}

template <typename VT, int LB>
static hipError_t launch_merge_rc(const CDev& p, int j, const void* in, void* out, dim3 grid,
                                  int threads, size_t lds, hipStream_t s) {
    if (p.R <= 8)
        hipLaunchKernelGGL((c_merge_kernel<VT, LB, 8>), grid, dim3(threads), lds, s, p, j, in, out);
    else if (p.R <= 16)
        hipLaunchKernelGGL((c_merge_kernel<VT, LB, 16>), grid, dim3(threads), lds, s, p, j, in, out);
    else if (p.R <= 24)
        hipLaunchKernelGGL((c_merge_kernel<VT, LB, 24>), grid, dim3(threads), lds, s, p, j, in, out);
    else
        hipLaunchKernelGGL((c_merge_kernel<VT, LB, 32>), grid, dim3(threads), lds, s, p, j, in, out);
    return hipGetLastError();
}

template <typename VT>
static hipError_t launch_merge_lb(const CDev& p, int j, const void* in, void* out, int lb,
                                  dim3 grid, int threads, size_t lds, hipStream_t s) {
    if (lb == 32) return launch_merge_rc<VT, 32>(p, j, in, out, grid, threads, lds, s);
    if (lb == 16) return launch_merge_rc<VT, 16>(p, j, in, out, grid, threads, lds, s);
    if (lb == 12) return launch_merge_rc<VT, 12>(p, j, in, out, grid, threads, lds, s);
    if (lb == 8) return launch_merge_rc<VT, 8>(p, j, in, out, grid, threads, lds, s);
    return launch_merge_rc<VT, 4>(p, j, in, out, grid, threads, lds, s);
}

// One merge launch of level j at block width lb (the launch_c_chain arithmetic).
template <typename VT>
static hipError_t launch_merge_once(const CDev& p, int j, int lb, hipStream_t s) {
    const int64_t nlo = p.pow_r[j - 1];
    const int64_t nlob = (nlo + lb - 1) / lb;
    const int64_t nhi = p.nblk / (nlo * p.R);
    const int threads = ((p.R * lb + 63) / 64) * 64;
    const int64_t nwg = nhi * nlob * p.P * p.R;
    if (nwg > 0x7fffffff || nlo * p.R > 0x7fffffff || p.R > 32 ||
        c_lds_for<VT>(p, lb) > 65536 || p.R * lb > 1024)
        return hipErrorInvalidConfiguration;
    return launch_merge_lb<VT>(p, j, p.t0, p.t1, lb, dim3((unsigned)nwg), threads,
                               c_lds_for<VT>(p, lb), s);
}

// One launch of level j at block width lb as a sweep runs it: the fused top merge and
// final sum for the top level of the order-independent case (values into t1, read and
// written in place by each lane), else the merge kernel from t0 into t1.
template <typename VT>
static hipError_t launch_level_once(const CDev& p, int j, int lb, hipStream_t s) {
    if (j == p.m - 1 && p.exogenous) {
        CDev q = p;
        q.v_in = p.t1;
        q.v_out = p.t1;
        return launch_top_final<VT>(q, p.t0, lb, s);
    }
    if (j == 3 && p.m >= 5) {
        // level 3 runs fused with level 2 where it fits; otherwise the first merge is
        // timed with it, so that every width is timed on the same work
        if (c_use23<VT>(p, lb)) return launch_merge23<VT>(p, p.u, p.t1, lb, s);
        hipError_t e = launch_c_chain<VT>(p, nullptr, 2, s);  // U into t0
        if (e != hipSuccess) return e;
    }
    return launch_merge_once<VT>(p, j, lb, s);
}

template <typename VT>
static hipError_t tune_levels(const CDev& p, hipStream_t s, int32_t* lb_out) {
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return e;
    }
    for (int j = 3; j <= p.m - 1 && j < 10 && e == hipSuccess; ++j) {
        float best = 1e30f;
        const bool fused = j == p.m - 1 && p.exogenous;
        for (int lb : {4, 8, 12, 16, 32}) {
            const bool fits = c_lds_for<VT>(p, lb) <= 65536 &&
                              p.R * lb <= (fused ? kCFusedThreads : 1024);
            if (!fits && !(j == 3 && c_use23<VT>(p, lb))) continue;
            if ((e = launch_level_once<VT>(p, j, lb, s)) != hipSuccess) break;  // warm-up
            if ((e = hipEventRecord(e0, s)) != hipSuccess) break;
            for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch_level_once<VT>(p, j, lb, s);
            if (e != hipSuccess || (e = hipEventRecord(e1, s)) != hipSuccess ||
                (e = hipEventSynchronize(e1)) != hipSuccess)
                break;
            float ms = 0.f;
            if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
            if (ms < best) {
                best = ms;
                lb_out[j] = lb;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return e;
}

hipError_t tune_c_merge(const CDev& pin, hipStream_t s, int32_t lb[2][10]) {
    CDev p = pin;
    p.extract = 1;  // the merge kernels then ignore the stop flag
    p.alim = p.R - 1;
    p.top_only = 0;
    for (int v = 0; v < 2; ++v)
        for (int j = 0; j < 10; ++j) lb[v][j] = 0;
    if (p.m < 4) return hipSuccess;  // no level j >= 3
    hipError_t e = tune_levels<double>(p, s, lb[0]);
    if (e == hipSuccess) e = tune_levels<float>(p, s, lb[1]);
    return e;
}

hipError_t launch_backup_c(const CDev& p, int storage_fp32, int extract, hipStream_t s) {
    if (extract) return launch_c_t<double, true>(p, s);
    if (storage_fp32) return launch_c_t<float, false>(p, s);
    return launch_c_t<double, false>(p, s);
}

}  // namespace pvi
