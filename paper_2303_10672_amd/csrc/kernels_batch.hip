// Value iteration of small scenario-A instances, one work group per instance, served
// by a persistent slot kernel that the host refills while it runs.
//
// One work group solves one instance completely (solve_item): both value tables live
// in LDS, the work group sweeps (deterministic-transition update of Methods, "Value
// iteration"; T from Appendix A), reduces max/min of V_new - V itself, applies the
// span stopping rule, and finally extracts the greedy policy with one more FP64
// backup.  The FP32 schedule keeps V in LDS as centred FP32 (V = c + v) until the
// span reaches the FP32 floor, then converts to FP64 and polishes to the threshold.
// Every instance has its own sizes, costs and tables; each work group's arithmetic
// depends only on its own instance, which makes results independent of what else
// runs.  The sweep loop is bounded by max_sweeps, so every solve ends.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "device_common.h"
#include "pvi_internal.h"
#include "slot_layout.h"

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

// The whole solve of one instance by one work group (256 threads): tables into LDS,
// the FP32 phase (FP32 schedule), the FP64 phase, the extraction, results to it.v,
// it.pi, it.gap, it.stats.
template <int RMAX>
__device__ void solve_item(const BatchItem& it, unsigned char* smem, double* red,
                           BatchShared& sh) {
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

// The slot kernel: work group k serves slot k of the table for as long as the host
// keeps it alive.  It waits for the slot's request number to move past the last one
// it served, copies the request's descriptor into LDS with system-coherent loads (the
// host rewrites the slot for every request, so nothing of it may come from a cache),
// solves it with solve_item, makes its results visible to the host and then publishes
// the request number as done.  With no request pending it returns when the host has
// set the stop word, or when the heartbeat word has not changed for kSlotIdlePolls
// polls (a host that stopped serving), so every work group ends.  The poll interval
// backs off from about 3 us to about 27 us while the slot is idle.  The work group
// size (64, 128 or 256 threads) is a launch parameter: solve_item strides over the
// states by the block size and reduces over whole wavefronts, so the results do not
// depend on it.
__device__ __forceinline__ uint32_t load_sys(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <int RMAX>
__global__ __launch_bounds__(256) void slot_kernel(SlotHeader* hdr, SlotSync* sync,
                                                   const BatchItem* items) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[64];
    __shared__ BatchShared sh;
    __shared__ uint32_t s_item[(sizeof(BatchItem) + 3) / 4];
    __shared__ uint32_t s_seq;
    __shared__ int s_exit;
    const int k = blockIdx.x;
    uint32_t last = 0;
    if (threadIdx.x == 0) last = load_sys(&sync[k].done);
    for (;;) {
        if (threadIdx.x == 0) {
            uint32_t hb_seen = load_sys(&hdr->heartbeat), still = 0, s = last;
            int nap = 1, ex = 0;
            for (;;) {
                // a request already in the slot is served even when the stop word is set
                s = load_sys(&sync[k].seq);
                if (s != last) break;
                if (load_sys(&hdr->stop)) {
                    ex = 1;
                    break;
                }
                const uint32_t hb = load_sys(&hdr->heartbeat);
                if (hb != hb_seen) {
                    hb_seen = hb;
                    still = 0;
                } else if (++still > kSlotIdlePolls) {
                    ex = 1;
                    break;
                }
                for (int i = 0; i < nap; ++i) __builtin_amdgcn_s_sleep(127);
                nap = nap < 8 ? 2 * nap : 8;
            }
            s_exit = ex;
            s_seq = s;
        }
        __syncthreads();
        if (s_exit) return;
        __atomic_thread_fence(__ATOMIC_ACQUIRE);
        const uint32_t* src = reinterpret_cast<const uint32_t*>(items + k);
        for (int i = threadIdx.x; i < (int)((sizeof(BatchItem) + 3) / 4); i += blockDim.x)
            s_item[i] = load_sys(src + i);
        __syncthreads();
        BatchItem it;
        __builtin_memcpy(&it, s_item, sizeof(BatchItem));
        solve_item<RMAX>(it, smem, red, sh);
        // every thread's result writes reach host memory before the slot is marked done
        __threadfence_system();
        __syncthreads();
        if (threadIdx.x == 0) {
            __hip_atomic_store(&sync[k].done, s_seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            last = s_seq;
        }
    }
}

hipError_t launch_slots(SlotHeader* hdr, SlotSync* sync, const BatchItem* items, int nslots,
                        int threads, size_t lds_bytes, hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    if (lds_bytes > 65536 - 1024 || (threads != 64 && threads != 128 && threads != 256))
        return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((slot_kernel<kSlotRmax>), dim3(nslots), dim3(threads), lds_bytes, s, hdr,
                       sync, items);
    return hipGetLastError();
}

int slot_capacity(int threads, size_t lds_bytes) {
    int dev = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(&slot_kernel<kSlotRmax>), threads,
            lds_bytes) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * cus;
}

}  // namespace pvi
