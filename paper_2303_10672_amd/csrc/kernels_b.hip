// Scenario B (two products, one-way substitution, L = 0) Bellman backup.
//
// Follows the deterministic-transition update (Methods, "Value iteration") with
// T from Appendix B (two-product FIFO equation, reward equation) and the
// substitution rule of the Scenario B description, in the direction "unmet demand
// of product 0 may take product 1": k ~ Binomial(u0, rho) of the u0 unmet
// product-0 customers are served from product-1 stock left after product 1's own
// demand, oldest first.
//
// Two facts shape the kernel:
//  * Product 1 sees the total demand e = d1 + k, so its outcome distribution given
//    u0 is E[u0][e] = sum_k Bin(k; u0, rho) P1(e - k) (a host table).  Its next
//    stock and revenue depend on e only.
//  * Product 0's next stock is zero whenever u0 > 0.
// Stage 1 therefore tabulates, for every product-0 next index i0' (with u0 = 0)
// and for i0' = 0 with each u0 >= 1 ("rows"), and every product-1 part
// (stock digits, order a1) ("cols"):
//     Z[row][col] = c_rev1 E_u[min(e, stock1)] + gamma sum_e E[u][e] V[i0', i1'(e)]
// with the FIFO-path form of the product-1 sum (demand up to the oldest stock
// leaves the younger units untouched; beyond it, k more units deplete them).
// Stage 2, one workgroup per product-1 stock index, sums the product-0 demand:
//     Q(s, a0, a1) = -c_var.a + c_rev0 E[min(d0, stock0)] + sum_d0 P0(d0) Z[row(d0)][col]
// and takes the max over the joint actions (a0 major, lowest index on ties).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>

#include "device_common.h"
#include "pvi_internal.h"

namespace pvi {

template <typename VT>
__global__ __launch_bounds__(256) void subst_stage1_kernel(BDev p) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p.ctl->stop && !p.extract) return;
    const int64_t ncol = (int64_t)p.nb * p.r1;
    if (idx >= (int64_t)p.rows * ncol) return;
    const int row = (int)(idx / ncol);
    const int col = (int)(idx - (int64_t)row * ncol);
    const int i0n = row < p.na ? row : 0;          // next product-0 index
    const int u = row < p.na ? 0 : row - p.na + 1;  // unmet product-0 demand
    const int ib = col / p.r1, a1 = col - ib * p.r1;
    // product-1 stock by remaining life: v[1] = B_2 .. v[m-2] = B_{m-1}, v[m-1] = a1
    int v[8];
    int rest = ib;
    const int x1 = rest % p.r1;  // B_1, the oldest
    rest /= p.r1;
    int K = 0;
    for (int j = 1; j <= p.m - 2; ++j) {
        v[j] = rest % p.r1;
        rest /= p.r1;
        K += v[j];
    }
    v[p.m - 1] = a1;
    K += a1;
    const double* Pu = p.e_pmf + (size_t)u * p.ew;
    const double* Fu = p.e_cdf + (size_t)u * p.ew;
    const double* Gu = p.e_tail + (size_t)u * p.ew;
    const VT* V = reinterpret_cast<const VT*>(p.v_in) + (int64_t)i0n * p.nb;
    double acc = 0.0;
    const int kmax = K == 0 ? 0 : max(0, min(K, p.emax - x1));
    for (int k = 0; k <= kmax; ++k) {
        const double w = K == 0 ? 1.0 : k == 0 ? Fu[min(x1, p.emax)] : k == K ? Gu[x1 + K]
                                                                             : Pu[x1 + k];
        // deplete the younger units by k, oldest first; life j+1 becomes digit j
        int r = k, off = 0, pw = 1;
        for (int j = 1; j <= p.m - 1; ++j) {
            const int take = min(r, v[j]);
            r -= take;
            off += (v[j] - take) * pw;
            pw *= p.r1;
        }
        acc = fma(w, (double)V[off], acc);
    }
    const int stock1 = x1 + K;
    p.z[idx] = p.rexp1[(size_t)u * p.sw + stock1] + p.gamma * acc;
}

// Merge two (best, second, argmax) triples; equal values go to the lower action.
__device__ __forceinline__ void merge_best(double& b, double& s2, int& a, double ob, double os,
                                           int oa) {
    const bool take = ob > b || (ob == b && oa < a);
    s2 = fmax(fmin(b, ob), fmax(s2, os));
    if (take) {
        b = ob;
        a = oa;
    }
}

// Stage 2: one workgroup per product-1 stock index; four neighbouring lanes share a
// product-0 stock index and split its orders a0 (a0 = part, part + 4, ...), then
// merge their best actions with two shuffles.
template <typename VT, bool EXTRACT>
__global__ __launch_bounds__(1024) void subst_stage2_kernel(BDev p) {
    extern __shared__ __align__(16) unsigned char smem[];
    if (!EXTRACT && p.ctl->stop) return;
    constexpr int NP = 4;
    const int ib = blockIdx.x, tid = threadIdx.x;
    const int R1 = p.r1, RP = p.r1pad;
    double* Zs = reinterpret_cast<double*>(smem);          // [rows][RP]
    double* P0 = Zs + (size_t)p.rows * RP;                  // [d0max+1]
    double* red = P0 + (p.d0max + 1);
    for (int i = tid; i < p.rows * RP; i += blockDim.x) {
        const int row = i / RP, a1 = i - row * RP;
        Zs[i] = a1 < R1 ? p.z[(int64_t)row * p.nb * R1 + (int64_t)ib * R1 + a1] : 0.0;
    }
    for (int i = tid; i <= p.d0max; i += blockDim.x) P0[i] = p.pmf0[i];
    __syncthreads();
    const double mu = (!EXTRACT && sizeof(VT) == 4) ? p.ctl->mu : 0.0;
    const int part = tid % NP, cells = blockDim.x / NP;
    double dmx = -DBL_MAX, dmn = DBL_MAX, vmx = -DBL_MAX, vmn = DBL_MAX;
    for (int ia0 = 0; ia0 < p.na; ia0 += cells) {   // same trip count on every lane
        const int ia = ia0 + tid / NP;
        const bool active = ia < p.na;
        double best = -DBL_MAX, second = -DBL_MAX;
        int arg = 0x7fffffff;
        if (active) {
            // product-0 stock by life: x0 = A_1 (oldest), w[1..m-2] = A_2..A_{m-1}
            int w[8];
            int rest = ia;
            const int x0 = rest % p.r0;
            rest /= p.r0;
            int held = x0;
            for (int j = 1; j <= p.m - 2; ++j) {
                w[j] = rest % p.r0;
                rest /= p.r0;
                held += w[j];
            }
            for (int a0 = part; a0 < p.r0; a0 += NP) {
                w[p.m - 1] = a0;
                const int stock0 = held + a0;
                double acc[PVI_B_R1MAX];
#pragma unroll
                for (int i = 0; i < PVI_B_R1MAX; ++i) acc[i] = 0.0;
                for (int d0 = 0; d0 <= p.d0max; ++d0) {
                    const double pr = P0[d0];
                    int row;
                    if (d0 >= stock0) {
                        row = d0 == stock0 ? 0 : p.na + (d0 - stock0) - 1;
                    } else {
                        // demand beyond the oldest units depletes the younger ones
                        int r = d0 > x0 ? d0 - x0 : 0, off = 0, pw = 1;
                        for (int j = 1; j <= p.m - 1; ++j) {
                            const int take = min(r, w[j]);
                            r -= take;
                            off += (w[j] - take) * pw;
                            pw *= p.r0;
                        }
                        row = off;
                    }
                    const double2* zr = reinterpret_cast<const double2*>(Zs + (size_t)row * RP);
#pragma unroll
                    for (int i = 0; i < PVI_B_R1MAX / 2; ++i) {
                        const double2 z = zr[i];
                        acc[2 * i] = fma(pr, z.x, acc[2 * i]);
                        acc[2 * i + 1] = fma(pr, z.y, acc[2 * i + 1]);
                    }
                }
                // the order costs as explicit fused multiply-adds, so that no kernel
                // depends on how the compiler contracts them
                const double base = fma(-p.cvar0, (double)a0, p.rexp0[stock0]);
#pragma unroll
                for (int a1 = 0; a1 < PVI_B_R1MAX; ++a1) {
                    if (a1 < R1) {
                        const double q = fma(-p.cvar1, (double)a1, base) + acc[a1];
                        if (q > best) {
                            second = best;
                            best = q;
                            arg = a0 * R1 + a1;
                        } else if (q > second) {
                            second = q;
                        }
                    }
                }
            }
        }
        for (int o = 1; o < NP; o <<= 1) {
            const double ob = __shfl_xor(best, o, 64);
            const double os = __shfl_xor(second, o, 64);
            const int oa = __shfl_xor(arg, o, 64);
            merge_best(best, second, arg, ob, os, oa);
        }
        if (!active || part != 0) continue;
        const int64_t s = (int64_t)ia * p.nb + ib;
        if (EXTRACT) {
            p.pi[s] = arg;
            p.gap[s] = best - second;
        } else {
            const VT o = (VT)(best - mu);
            reinterpret_cast<VT*>(p.v_out)[s] = o;
            const double out = (double)o;
            const double dv = out - (double)reinterpret_cast<const VT*>(p.v_in)[s];
            dmx = fmax(dmx, dv);
            dmn = fmin(dmn, dv);
            vmx = fmax(vmx, out);
            vmn = fmin(vmn, out);
        }
    }
    if (EXTRACT) return;
    block_reduce4(dmx, dmn, vmx, vmn, red);
    if (tid == 0) {
        double* pp = p.partials + 4 * (size_t)ib;
        pp[0] = dmx;
        pp[1] = dmn;
        pp[2] = vmx;
        pp[3] = vmn;
    }
}

// Pointer into the constant address space: loads through it whose address is the
// same for every lane go through the scalar cache.
typedef const __attribute__((address_space(4))) double* ConstF64B;

constexpr int kBX = 16;  // oldest-digit sums per lane in the tiled kernels (R0, R1 <= 16)

// Depletes k units from the younger digits v[1..m-1] oldest first and returns the
// offset of what is left (digit j weighs radix^(j-1)).
// M > 0: m known at compile time (no per-digit branches).
template <int M = 0>
__device__ __forceinline__ int b_path_offset(const int (&v)[8], int m, int radix, int k) {
    int r = k, off = 0, pw = 1;
#pragma unroll
    for (int j = 1; j < (M > 0 ? M : 8); ++j) {
        if (M > 0 || j <= m - 1) {
            const int take = min(r, v[j]);
            r -= take;
            off += (v[j] - take) * pw;
            pw *= radix;
        }
    }
    return off;
}

// Stage 1, tiled: one wavefront per (row, four middle-digit indices bi of product
// 1), lane (slot, a1).  A lane walks the FIFO path of its younger digits
// (B_2..B_{m-1}, a1) once and keeps one sum per oldest digit x1, so every value read
// from V serves all x1; the weights P_u(x1 + k) of the points before the path's end
// do not depend on the lane and come through the scalar cache.  Per cell the terms
// and their order are those of subst_stage1_kernel; the terms that kernel skips
// (total demand beyond emax) enter here with weight zero, which leaves every sum
// unchanged.
template <typename VT, int KB, int M>
__global__ __launch_bounds__(64) void subst_stage1_tiled_kernel(BDev p) {
    if (p.ctl->stop && !p.extract) return;
    const int R1 = p.r1, m = M > 0 ? M : p.m;
    const int nbi = p.nb / R1;  // middle digits B_2..B_{m-1}
    const int nq = (nbi + 3) >> 2;
    const int row = blockIdx.x / nq, q = blockIdx.x - row * nq;
    const int lane = threadIdx.x, a1l = lane & 15, bil = q * 4 + (lane >> 4);
    // lanes past the orders or the digit range repeat a real cell and store nothing
    const bool live = a1l < R1 && bil < nbi;
    const int a1 = min(a1l, R1 - 1), bi = min(bil, nbi - 1);
    const int i0n = row < p.na ? row : 0;
    const int u = row < p.na ? 0 : row - p.na + 1;
    int v[8];
    int K = 0;
    {
        int rest = bi;
#pragma unroll
        for (int j = 1; j < 8; ++j) {
            if (j <= m - 2) {
                v[j] = rest % R1;
                rest /= R1;
            } else {
                v[j] = j == m - 1 ? a1 : 0;
            }
            K += v[j];
        }
    }
    const VT* Vr = reinterpret_cast<const VT*>(p.v_in) + (int64_t)i0n * p.nb;
    const ConstF64B Fu = (ConstF64B)(p.e_cdf + (size_t)u * p.ew);
    const ConstF64B Pu = (ConstF64B)(p.ppad + (size_t)u * p.ewp);
    const double* Gu = p.gpad + (size_t)u * p.ewp;
    auto load = [&](int k) { return (double)Vr[b_path_offset<M>(v, m, R1, k)]; };

    double acc[kBX];
    {
        const double v0 = load(0);
#pragma unroll
        for (int x1 = 0; x1 < kBX; ++x1) {
            acc[x1] = 0.0;
            const double w = K == 0 ? 1.0 : Fu[min(x1, p.emax)];
            acc[x1] = fma(w, v0, acc[x1]);
        }
    }
    auto step = [&](int k, double vk) {
        if (k < K) {
#pragma unroll
            for (int x1 = 0; x1 < kBX; ++x1) acc[x1] = fma(Pu[x1 + k], vk, acc[x1]);
        }
    };
    if constexpr (KB > 0) {
        // points 1 .. K - 1 with K < KB: every value of the path is loaded before the
        // first is used (any k gives an offset inside the row), so a wavefront waits
        // for memory once
        double pv[KB];
#pragma unroll
        for (int k = 1; k < KB; ++k) pv[k] = load(k);
#pragma unroll
        for (int k = 1; k < KB; ++k) step(k, pv[k]);
    } else {
        // longer paths: up to the wavefront's longest, values loaded four points ahead
        const int kw = (int)wave_max((double)K);
        double va = load(1), vb = load(2), vc = load(3), vd = load(4);
        for (int k = 1; k < kw; k += 4) {
            step(k, va);
            va = load(k + 4);
            if (k + 1 >= kw) break;
            step(k + 1, vb);
            vb = load(k + 5);
            if (k + 2 >= kw) break;
            step(k + 2, vc);
            vc = load(k + 6);
            if (k + 3 >= kw) break;
            step(k + 3, vd);
            vd = load(k + 7);
        }
    }
    // the path's end: every younger unit gone, weight P_u(e >= x1 + K)
    if (K > 0) {
        const double vK = (double)Vr[0];
#pragma unroll
        for (int x1 = 0; x1 < kBX; ++x1) acc[x1] = fma(Gu[x1 + K], vK, acc[x1]);
    }
    if (!live) return;
    double* zr = p.z + (int64_t)row * p.nb * R1 + (int64_t)bi * R1 * R1 + a1;
    const double* rx = p.rexp1 + (size_t)u * p.sw + K;
#pragma unroll
    for (int x1 = 0; x1 < kBX; ++x1)
        if (x1 < R1) zr[x1 * R1] = rx[x1] + p.gamma * acc[x1];
}

// Stage 2, tiled: one workgroup per (product-1 stock index ib, middle product-0 digits
// w); lane (a0, a1) of a 16 x 16 grid.  With the younger product-0 digits (w, a0)
// fixed, product-0 demand x0 + j lands on point j of one list of Z rows for every
// oldest digit x0 (j <= K depletes the younger units, beyond it j - K units are
// unmet), so a lane loads the Z entries of its column a1 at those points once and
// forms the sums of all x0 from them.  Each sum takes its terms in the order of
// subst_stage2_kernel (d0 ascending), so the values are the same; the maximum over
// a1 is a 16-lane transpose-reduction, over a0 one over four lane groups and the
// four wavefronts.
template <typename VT, int J, bool EXTRACT>
__global__ __launch_bounds__(256) void subst_stage2_tiled_kernel(BDev p) {
    constexpr int TS = kBX + 2;  // row stride of the Q tile (16-byte rows, spread banks)
    __shared__ int32_t roff[kBX * J];
    __shared__ __align__(16) double qt[kBX * kBX * TS];  // [a0][a1][x0]
    __shared__ double red[4 * kBX];
    __shared__ double red2[EXTRACT ? 4 * kBX : 1];
    __shared__ int32_t reda[EXTRACT ? 4 * kBX : 1];
    if (!EXTRACT && p.ctl->stop) return;
    const int grp = xcd_remap(blockIdx.x, gridDim.x);
    const int ib = grp / p.nw, wi = grp - ib * p.nw;
    const int R0 = p.r0, R1 = p.r1, m = p.m, tid = threadIdx.x;
    // middle product-0 digits w[1..m-2] = A_2..A_{m-1}
    int w[8];
    int held = 0;
    {
        int rest = wi;
#pragma unroll
        for (int j = 1; j < 8; ++j) {
            w[j] = 0;
            if (j <= m - 2) {
                w[j] = rest % R0;
                rest /= R0;
            }
            held += w[j];
        }
    }
    // element offset of the Z row at point j of tile a0 (rows of nb * R1 entries)
    const int zrow = p.nb * R1;
    for (int e = tid; e < kBX * J; e += blockDim.x) {
        const int t = e / J, j = e - t * J;
        int row = 0;
        if (t < R0 && j <= p.d0max) {
            const int K = held + t;
            if (j <= K) {
                int v[8];
#pragma unroll
                for (int d = 1; d < 8; ++d) v[d] = d == m - 1 ? t : w[d];
                row = b_path_offset(v, m, R0, j);
            } else {
                row = p.na + (j - K) - 1;
            }
        }
        roff[e] = row * zrow;
    }
    __syncthreads();

    const int wv = tid >> 6, l16 = tid & 15;
    const int a0 = min(wv * 4 + ((tid >> 4) & 3), R0 - 1), a1 = min(l16, R1 - 1);
    const double* zc = p.z + (int64_t)ib * R1 + a1;
    double zr[J];
#pragma unroll
    for (int j = 0; j < J; ++j) zr[j] = zc[roff[a0 * J + j]];

    // demand values past d0max (up to J) add terms of weight zero, which leave the
    // sums unchanged
    const ConstF64B P0 = (ConstF64B)p.pmf0;
    const int d0max = p.d0max;
    double acc[kBX];
#pragma unroll
    for (int x0 = 0; x0 < kBX; ++x0) acc[x0] = 0.0;
#pragma unroll
    for (int d0 = 0; d0 < J; ++d0) {
        const double pr = d0 <= d0max ? P0[min(d0, d0max)] : 0.0;
#pragma unroll
        for (int x0 = 0; x0 < kBX; ++x0) acc[x0] = fma(pr, zr[d0 > x0 ? d0 - x0 : 0], acc[x0]);
    }
    // lanes past the orders repeat the Q values of a real action, which leaves every
    // maximum unchanged (policy extraction, which also needs the second best, gives
    // them -DBL_MAX); entries x0 >= R0 are not states and are never stored.  The Q
    // values go to LDS as [a0][a1][x0]; thread (a0, x0) then takes the maximum over
    // a1, and over a0 two lane exchanges and the four wavefronts follow.
    const bool real = wv * 4 + ((tid >> 4) & 3) < R0 && l16 < R1;
    {
        double2* row = reinterpret_cast<double2*>(qt + (size_t)(tid >> 4) * kBX * TS + l16 * TS);
#pragma unroll
        for (int x0 = 0; x0 < kBX; x0 += 2) {
            const double q0 = fma(-p.cvar1, (double)a1,
                                  fma(-p.cvar0, (double)a0, p.rexp0[min(x0, R0 - 1) + held + a0])) +
                              acc[x0];
            const double q1 = fma(-p.cvar1, (double)a1,
                                  fma(-p.cvar0, (double)a0,
                                      p.rexp0[min(x0 + 1, R0 - 1) + held + a0])) +
                              acc[x0 + 1];
            row[x0 / 2] = EXTRACT && !real ? make_double2(-DBL_MAX, -DBL_MAX) : make_double2(q0, q1);
        }
    }
    __syncthreads();
    if constexpr (EXTRACT) {
        // (best, second, argmax) with ties to the lowest action a0 R1 + a1, as the
        // per-state kernel takes them
        const int a0s = tid >> 4;
        const double* col = qt + (size_t)a0s * kBX * TS + l16;
        double best = -DBL_MAX, second = -DBL_MAX;
        int arg = 0x7fffffff;
#pragma unroll
        for (int i = 0; i < kBX; ++i) {
            const double q = col[i * TS];
            if (q > best) {
                second = best;
                best = q;
                arg = a0s * R1 + i;
            } else if (q > second) {
                second = q;
            }
        }
        for (int o = 16; o <= 32; o <<= 1) {
            const double ob = __shfl_xor(best, o, 64);
            const double os = __shfl_xor(second, o, 64);
            const int oa = __shfl_xor(arg, o, 64);
            merge_best(best, second, arg, ob, os, oa);
        }
        if ((tid & 63) < kBX) {
            red[wv * kBX + l16] = best;
            red2[wv * kBX + l16] = second;
            reda[wv * kBX + l16] = arg;
        }
        __syncthreads();
        if (tid < R0) {
            double b = red[tid], s2 = red2[tid];
            int a = reda[tid];
            for (int w2 = 1; w2 < 4; ++w2)
                merge_best(b, s2, a, red[w2 * kBX + tid], red2[w2 * kBX + tid], reda[w2 * kBX + tid]);
            const int64_t st = (int64_t)(tid + R0 * wi) * p.nb + ib;
            p.pi[st] = a;
            p.gap[st] = b - s2;
        }
        return;
    }
    double best;
    {
        const double* col = qt + (size_t)(tid >> 4) * kBX * TS + l16;
        best = col[0];
#pragma unroll
        for (int i = 1; i < kBX; ++i) best = fmax(best, col[i * TS]);
    }
    best = fmax(best, __shfl_xor(best, 16, 64));
    best = fmax(best, __shfl_xor(best, 32, 64));
    if ((tid & 63) < kBX) red[wv * kBX + l16] = best;
    __syncthreads();
    if (tid >= 64) return;
    const double mu = sizeof(VT) == 4 ? p.ctl->mu : 0.0;
    double dmx = -DBL_MAX, dmn = DBL_MAX, vmx = -DBL_MAX, vmn = DBL_MAX;
    if (tid < R0) {
        const double b = fmax(fmax(red[tid], red[kBX + tid]), fmax(red[2 * kBX + tid], red[3 * kBX + tid]));
        const int64_t s = (int64_t)(tid + R0 * wi) * p.nb + ib;
        const VT o = (VT)(b - mu);
        reinterpret_cast<VT*>(p.v_out)[s] = o;
        const double out = (double)o;
        const double dv = out - (double)reinterpret_cast<const VT*>(p.v_in)[s];
        dmx = dv;
        dmn = dv;
        vmx = out;
        vmn = out;
    }
    dmx = wave_max(dmx);
    dmn = wave_min(dmn);
    vmx = wave_max(vmx);
    vmn = wave_min(vmn);
    if (tid == 0) {
        double* pp = p.partials + 4 * (size_t)grp;
        pp[0] = dmx;
        pp[1] = dmn;
        pp[2] = vmx;
        pp[3] = vmn;
    }
}

template <typename VT, bool EXTRACT>
static hipError_t launch_b_t(const BDev& p, hipStream_t s) {
    if (p.tiled) {
        const dim3 grid1((unsigned)(p.rows * ((p.nb / p.r1 + 3) / 4)));
        // paths of at most (m - 1)(R1 - 1) younger units: loaded whole when that fits
        const int kmax = (p.m - 1) * (p.r1 - 1);
        // the two- and three-digit shapes (m = 2, 3) have their own instances
        if (kmax < 16 && p.m == 2)
            hipLaunchKernelGGL((subst_stage1_tiled_kernel<VT, 16, 2>), grid1, dim3(64), 0, s, p);
        else if (kmax < 32 && p.m == 3)
            hipLaunchKernelGGL((subst_stage1_tiled_kernel<VT, 32, 3>), grid1, dim3(64), 0, s, p);
        else if (kmax < 16)
            hipLaunchKernelGGL((subst_stage1_tiled_kernel<VT, 16, 0>), grid1, dim3(64), 0, s, p);
        else if (kmax < 32)
            hipLaunchKernelGGL((subst_stage1_tiled_kernel<VT, 32, 0>), grid1, dim3(64), 0, s, p);
        else
            hipLaunchKernelGGL((subst_stage1_tiled_kernel<VT, 0, 0>), grid1, dim3(64), 0, s, p);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const dim3 grid((unsigned)(p.nb * p.nw));
        // the fewest demand values J >= d0max + 1 of the compiled widths
        if (p.d0max < 8)
            hipLaunchKernelGGL((subst_stage2_tiled_kernel<VT, 8, EXTRACT>), grid, dim3(256), 0, s, p);
        else if (p.d0max < 16)
            hipLaunchKernelGGL((subst_stage2_tiled_kernel<VT, 16, EXTRACT>), grid, dim3(256), 0, s,
                               p);
        else if (p.d0max == 20)  // demand folded at 20, the paper's truncation
            hipLaunchKernelGGL((subst_stage2_tiled_kernel<VT, 21, EXTRACT>), grid, dim3(256), 0, s,
                               p);
        else if (p.d0max < 24)
            hipLaunchKernelGGL((subst_stage2_tiled_kernel<VT, 24, EXTRACT>), grid, dim3(256), 0, s,
                               p);
        else
            hipLaunchKernelGGL((subst_stage2_tiled_kernel<VT, PVI_B_JMAX, EXTRACT>), grid, dim3(256),
                               0, s, p);
        return hipGetLastError();
    } else {
        const int64_t n1 = (int64_t)p.rows * p.nb * p.r1;
        hipLaunchKernelGGL((subst_stage1_kernel<VT>), dim3((unsigned)((n1 + 255) / 256)), dim3(256),
                           0, s, p);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const size_t bytes = sizeof(double) * ((size_t)p.rows * p.r1pad + p.d0max + 1 + 64);
    if (bytes > 65536) return hipErrorInvalidConfiguration;
    // four lanes per product-0 state; at most 1024 lanes
    const int threads = (int)std::min<int64_t>(1024, ((int64_t)p.na * 4 + 63) / 64 * 64);
    hipLaunchKernelGGL((subst_stage2_kernel<VT, EXTRACT>), dim3(p.nb), dim3(threads), bytes, s, p);
    return hipGetLastError();
}

hipError_t launch_backup_b(const BDev& p, int storage_fp32, int extract, hipStream_t s) {
    if (p.r1 > PVI_B_R1MAX) return hipErrorInvalidValue;
    if (extract) return launch_b_t<double, true>(p, s);
    if (storage_fp32) return launch_b_t<float, false>(p, s);
    return launch_b_t<double, false>(p, s);
}

}  // namespace pvi
