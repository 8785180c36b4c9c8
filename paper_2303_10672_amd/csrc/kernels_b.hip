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
                const double base = -p.cvar0 * a0 + p.rexp0[stock0];
#pragma unroll
                for (int a1 = 0; a1 < PVI_B_R1MAX; ++a1) {
                    if (a1 < R1) {
                        const double q = base - p.cvar1 * a1 + acc[a1];
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

template <typename VT, bool EXTRACT>
static hipError_t launch_b_t(const BDev& p, hipStream_t s) {
    const int64_t n1 = (int64_t)p.rows * p.nb * p.r1;
    hipLaunchKernelGGL((subst_stage1_kernel<VT>), dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0,
                       s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
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
