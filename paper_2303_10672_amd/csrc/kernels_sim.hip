// Rollouts of a replenishment policy (Simulation section: rollouts of warm-up plus
// counted days from a start state; the return is the discounted sum of the rewards
// of the counted days; the KPIs are the service level, the wastage and the
// holding), one lane per (policy, rollout) pair.
//
// Each lane keeps its stock by remaining life (and, for scenario A, its orders in
// transit) in registers, draws the day's randomness from Philox4x64-10 (Salmon,
// Moraes, Dror and Shaw, SC 2011) keyed by (seed, 0) with counter (rollout, day,
// block, 0), and applies the day's transition unit by unit: issue oldest first
// (youngest first for LIFO), discard what reaches the end of its life, age the
// rest, receive the arriving order.  Word 0 of block 0 is the demand of product
// 0, word 1 the demand of product 1; unit i of the day (a scenario-C unit's
// remaining life, a scenario-B customer's acceptance of substitution) uses word
// i%4 of block 1 + i/4.  Draws u = (x >> 11) 2^-53 become the smallest d with
// u < CDF(d) (d_max if none), the smallest life k with u < p_1 + .. + p_k (m if
// none), and acceptance when u < rho.  Every candidate policy sees the same
// numbers (common random numbers across a heuristic grid).
//
// The rollout is a chain of dependent days, so the kernel is latency bound: it
// runs thousands of independent lanes, keeps the demand CDFs in LDS, and reads
// the policy table with one 4-byte gather per day.  Floating-point contraction is
// off so the return is the plain sum of products of the definition.
#include <hip/hip_runtime.h>

#include "pvi_internal.h"

#pragma clang fp contract(off)

namespace pvi {

namespace {

constexpr int kMaxM = PVI_MAX_LIFE;  // life classes 1..m
constexpr int kMaxO = 11;            // orders in transit (scenario A, L - 1)
constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;

struct Block {
    uint64_t w[4];
};

__device__ __forceinline__ Block philox(uint64_t seed, uint64_t r, uint64_t t, uint64_t b) {
    uint64_t x0 = r, x1 = t, x2 = b, x3 = 0, k0 = seed, k1 = 0;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += kW0;
            k1 += kW1;
        }
        const uint64_t hi0 = __umul64hi(kM0, x0), lo0 = kM0 * x0;
        const uint64_t hi1 = __umul64hi(kM1, x2), lo1 = kM1 * x2;
        const uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
        x0 = y0;
        x1 = lo1;
        x2 = y2;
        x3 = lo0;
    }
    return Block{{x0, x1, x2, x3}};
}

// word j of a block by selects (a dynamic index would put the block in scratch)
__device__ __forceinline__ uint64_t word(const Block& b, int j) {
    const uint64_t lo = (j & 1) ? b.w[1] : b.w[0], hi = (j & 1) ? b.w[3] : b.w[2];
    return (j & 2) ? hi : lo;
}

__device__ __forceinline__ double unif(uint64_t x) {
    return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ int sample(const double* cdf, int dmax, double u) {
    int d = 0;
    while (d < dmax && !(u < cdf[d])) ++d;
    return d;
}

__device__ __forceinline__ double posd(double x) { return x > 0.0 ? x : 0.0; }

struct Tally {
    int demand, met, expired, received, held;
};

__device__ __forceinline__ void add(Tally& c, const Tally& d) {
    c.demand += d.demand;
    c.met += d.met;
    c.expired += d.expired;
    c.received += d.received;
    c.held += d.held;
}

// service %, wastage %, mean holding per day of a rollout's counts
__device__ __forceinline__ void kpis(double* k, const Tally& c, int horizon) {
    k[0] = c.demand > 0 ? 100.0 * (double)c.met / (double)c.demand : 100.0;
    k[1] = c.received > 0 ? 100.0 * (double)c.expired / (double)c.received : 0.0;
    k[2] = horizon > 0 ? (double)c.held / (double)horizon : 0.0;
}

}  // namespace

// FAM 0: scenario A (state [O_{L-1}..O_1, X_m..X_1]); 1: scenario B with L = 0
// ([A_{m-1}..A_1, B_{m-1}..B_1]); 2: scenario C ([tau, X_{m-1}..X_1]); 3: scenario B
// with lead time 1 ([Xa_m..Xa_1, Xb_m..Xb_1]; X holds product a, Y product b).
template <int FAM>
__global__ __launch_bounds__(64) void rollout_kernel(SimDev s) {
    extern __shared__ __align__(16) unsigned char smem[];
    double* cdf0 = reinterpret_cast<double*>(smem);
    double* cdf1 = cdf0 + s.n_cdf0;
    double* lcum = cdf1 + s.n_cdf1;
    for (int i = threadIdx.x; i < s.n_cdf0; i += blockDim.x) cdf0[i] = s.cdf0[i];
    for (int i = threadIdx.x; i < s.n_cdf1; i += blockDim.x) cdf1[i] = s.cdf1[i];
    for (int i = threadIdx.x; i < s.n_lcum; i += blockDim.x) lcum[i] = s.lifecum[i];
    __syncthreads();
    const int64_t lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= (int64_t)s.n_pol * s.n_roll) return;
    const int pol = (int)(lane / s.n_roll);
    const uint64_t r = (uint64_t)(lane - (int64_t)pol * s.n_roll);
    const int32_t* prm = s.params ? s.params + (size_t)pol * PVI_POLICY_PARAMS : nullptr;
    const int m = s.m, R0 = s.R0;

    // state registers; index 0 of X/B unused, lives 1..m
    int X[kMaxM + 1] = {}, Y[kMaxM + 1] = {}, O[kMaxO + 1] = {};
    int tau = 0;
    {
        int64_t idx = s.start;
        if (FAM == 0) {
#pragma unroll
            for (int j = 1; j <= kMaxM; ++j)  // X_1 is the least significant digit
                if (j <= m) {
                    X[j] = (int)(idx % R0);
                    idx /= R0;
                }
#pragma unroll
            for (int i = kMaxO; i >= 1; --i) O[i] = 0;
#pragma unroll
            for (int i = 1; i <= kMaxO; ++i)  // then O_1 .. O_{L-1}
                if (i <= s.L - 1) {
                    O[i] = (int)(idx % R0);
                    idx /= R0;
                }
        } else if (FAM == 1) {
#pragma unroll
            for (int j = 1; j < kMaxM; ++j)
                if (j <= m - 1) {
                    Y[j] = (int)(idx % s.R1);
                    idx /= s.R1;
                }
#pragma unroll
            for (int j = 1; j < kMaxM; ++j)
                if (j <= m - 1) {
                    X[j] = (int)(idx % R0);
                    idx /= R0;
                }
        } else if (FAM == 3) {
#pragma unroll
            for (int j = 1; j <= kMaxM; ++j)
                if (j <= m) {
                    Y[j] = (int)(idx % s.R1);
                    idx /= s.R1;
                }
#pragma unroll
            for (int j = 1; j <= kMaxM; ++j)
                if (j <= m) {
                    X[j] = (int)(idx % R0);
                    idx /= R0;
                }
        } else {
#pragma unroll
            for (int j = 1; j < kMaxM; ++j)
                if (j <= m - 1) {
                    X[j] = (int)(idx % R0);
                    idx /= R0;
                }
            tau = (int)idx;
        }
    }

    constexpr bool kTwo = FAM == 1 || FAM == 3;
    double g = 1.0, acc = 0.0;
    Tally c = {0, 0, 0, 0, 0};
    Tally c0 = {0, 0, 0, 0, 0}, c1 = {0, 0, 0, 0, 0};  // per product (two products)
    const int days = s.warmup + s.horizon;
    for (int t = 0; t < days; ++t) {
        // ---- action (two products: aA, aB; heuristic orders are not capped,
        // except scenario C's, whose remaining-life table ends at a_max)
        int a = 0, aA = 0, aB = 0;
        if (s.kind == PVI_POLICY_TABLE) {
            int64_t idx = 0;
            if (FAM == 0) {
#pragma unroll
                for (int i = kMaxO; i >= 1; --i)
                    if (i <= s.L - 1) idx = idx * R0 + O[i];
#pragma unroll
                for (int j = kMaxM; j >= 1; --j)
                    if (j <= m) idx = idx * R0 + X[j];
            } else if (FAM == 1) {
#pragma unroll
                for (int j = kMaxM - 1; j >= 1; --j)
                    if (j <= m - 1) idx = idx * R0 + X[j];
#pragma unroll
                for (int j = kMaxM - 1; j >= 1; --j)
                    if (j <= m - 1) idx = idx * s.R1 + Y[j];
            } else if (FAM == 3) {
#pragma unroll
                for (int j = kMaxM; j >= 1; --j)
                    if (j <= m) idx = idx * R0 + X[j];
#pragma unroll
                for (int j = kMaxM; j >= 1; --j)
                    if (j <= m) idx = idx * s.R1 + Y[j];
            } else {
                idx = tau;
#pragma unroll
                for (int j = kMaxM - 1; j >= 1; --j)
                    if (j <= m - 1) idx = idx * R0 + X[j];
            }
            a = s.table[idx];
            if (kTwo) {
                aA = a / s.R1;
                aB = a - aA * s.R1;
            }
        } else if (FAM == 0) {  // base stock on stock on hand and in transit
            int I = 0;
#pragma unroll
            for (int j = 1; j <= kMaxM; ++j) I += X[j];
#pragma unroll
            for (int i = 1; i <= kMaxO; ++i) I += O[i];
            a = max(prm[0] - I, 0);
        } else if (kTwo) {  // modified base stock per product
            int IA = 0, IB = 0;
#pragma unroll
            for (int j = 1; j <= kMaxM; ++j) {
                IA += X[j];
                IB += Y[j];
            }
            const double va = posd(((double)prm[0] - IA) + posd((double)X[1] - s.mu0));
            const double vb = posd(((double)prm[1] - IB) + posd((double)Y[1] - s.mu1));
            aA = (int)floor(va);
            aB = (int)floor(vb);
        } else {  // (s, S) of the weekday
            int I = 0;
#pragma unroll
            for (int j = 1; j < kMaxM; ++j) I += X[j];
            const int lo = prm[2 * tau], hi = prm[2 * tau + 1];
            a = (lo < hi && I <= lo) ? min(max(hi - I, 0), R0 - 1) : 0;
        }

        // ---- outcome and transition
        const Block b0 = philox(s.seed, r, (uint64_t)t, 0);
        double rew;
        Tally day, day0 = {0, 0, 0, 0, 0}, day1 = {0, 0, 0, 0, 0};
        if (FAM == 0) {
            const int d = sample(cdf0, s.dmax0, unif(b0.w[0]));
            int tot = 0;
#pragma unroll
            for (int j = 1; j <= kMaxM; ++j) tot += X[j];
            int rem = d;
            if (s.issuing == PVI_LIFO) {
#pragma unroll
                for (int j = kMaxM; j >= 1; --j) {
                    const int take = min(rem, X[j]);
                    X[j] -= take;
                    rem -= take;
                }
            } else {
#pragma unroll
                for (int j = 1; j <= kMaxM; ++j) {
                    const int take = min(rem, X[j]);
                    X[j] -= take;
                    rem -= take;
                }
            }
            const int met = d - rem, W = X[1];
            const int held = tot - met - W;
            rew = -s.cvar0 * a - s.chold * (double)held - s.cshort * (double)(d - met) -
                  s.cwaste * (double)W;
            const int arrive = s.L >= 2 ? O[1] : a;
#pragma unroll
            for (int j = 1; j < kMaxM; ++j) X[j] = j < m ? X[j + 1] : 0;
#pragma unroll
            for (int j = 1; j <= kMaxM; ++j)
                if (j == m) X[j] = arrive;
#pragma unroll
            for (int i = 1; i < kMaxO; ++i) O[i] = i < s.L - 1 ? O[i + 1] : 0;
#pragma unroll
            for (int i = 1; i <= kMaxO; ++i)
                if (i == s.L - 1) O[i] = a;
            day = Tally{d, met, W, arrive, held};
        } else if (FAM == 1) {
            const int dA = sample(cdf0, s.dmax0, unif(b0.w[0]));
            const int dB = sample(cdf1, s.dmax1, unif(b0.w[1]));
#pragma unroll
            for (int j = 1; j <= kMaxM; ++j)
                if (j == m) {
                    X[j] = aA;
                    Y[j] = aB;
                }
            int stA = 0, stB = 0;
#pragma unroll
            for (int j = 1; j <= kMaxM; ++j) {
                stA += X[j];
                stB += Y[j];
            }
            int rem = dA;
#pragma unroll
            for (int j = 1; j <= kMaxM; ++j) {
                const int take = min(rem, X[j]);
                X[j] -= take;
                rem -= take;
            }
            const int hA = dA - rem, unmet = rem;
            int k = 0;
            Block bu = b0;
            for (int i = 0; i < unmet; ++i) {
                if ((i & 3) == 0) bu = philox(s.seed, r, (uint64_t)t, (uint64_t)(1 + (i >> 2)));
                if (unif(word(bu, i & 3)) < s.rho) ++k;
            }
            rem = dB;
#pragma unroll
            for (int j = 1; j <= kMaxM; ++j) {
                const int take = min(rem, Y[j]);
                Y[j] -= take;
                rem -= take;
            }
            const int hB = dB - rem;
            rem = k;
#pragma unroll
            for (int j = 1; j <= kMaxM; ++j) {
                const int take = min(rem, Y[j]);
                Y[j] -= take;
                rem -= take;
            }
            const int hS = k - rem;
            const int wA = X[1], wB = Y[1], W = wA + wB;
            rew = -(s.cvar0 * aA + s.cvar1 * aB) + s.rev0 * hA + s.rev1 * (hB + hS);
#pragma unroll
            for (int j = 1; j < kMaxM; ++j) {
                X[j] = j < m ? X[j + 1] : 0;
                Y[j] = j < m ? Y[j + 1] : 0;
            }
            X[kMaxM] = Y[kMaxM] = 0;
            day = Tally{dA + dB, hA + hB + hS, W, aA + aB, stA + stB - hA - hB - hS - W};
            // product 0's customers served by product 1 count as met for product 0
            day0 = Tally{dA, hA + hS, wA, aA, stA - hA - wA};
            day1 = Tally{dB, hB, wB, aB, stB - hB - hS - wB};
        } else if (FAM == 3) {
            // lead time 1: today's orders arrive for tomorrow; product b's unmet
            // customers may take product a's units left after a's own demand
            const int dA = sample(cdf0, s.dmax0, unif(b0.w[0]));
            const int dB = sample(cdf1, s.dmax1, unif(b0.w[1]));
            int stA = 0, stB = 0;
#pragma unroll
            for (int j = 1; j <= kMaxM; ++j) {
                stA += X[j];
                stB += Y[j];
            }
            int rem = dB;
#pragma unroll
            for (int j = 1; j <= kMaxM; ++j) {
                const int take = min(rem, Y[j]);
                Y[j] -= take;
                rem -= take;
            }
            const int hB = dB - rem, excess = rem;
            int du = 0;
            Block bu = b0;
            for (int i = 0; i < excess; ++i) {
                if ((i & 3) == 0) bu = philox(s.seed, r, (uint64_t)t, (uint64_t)(1 + (i >> 2)));
                if (unif(word(bu, i & 3)) < s.rho) ++du;
            }
            rem = dA + du;
#pragma unroll
            for (int j = 1; j <= kMaxM; ++j) {
                const int take = min(rem, X[j]);
                X[j] -= take;
                rem -= take;
            }
            const int hA = dA + du - rem;
            const int wA = X[1], wB = Y[1], W = wA + wB;
            rew = -(s.cvar0 * aA + s.cvar1 * aB) + s.rev0 * hA + s.rev1 * hB;
#pragma unroll
            for (int j = 1; j < kMaxM; ++j) {
                X[j] = j < m ? X[j + 1] : 0;
                Y[j] = j < m ? Y[j + 1] : 0;
            }
            X[kMaxM] = Y[kMaxM] = 0;
#pragma unroll
            for (int j = 1; j <= kMaxM; ++j)
                if (j == m) {
                    X[j] = aA;
                    Y[j] = aB;
                }
            day = Tally{dA + dB, hA + hB, W, aA + aB, stA + stB - hA - hB - W};
            // product a's own customers come first; the rest of its issues went to
            // product b's customers and count as met for product b
            const int ownA = min(dA, stA);
            day0 = Tally{dA, ownA, wA, aA, stA - hA - wA};
            day1 = Tally{dB, hB + (hA - ownA), wB, aB, stB - hB - wB};
        } else {
            const int d = sample(cdf0 + tau * (s.dmax0 + 1), s.dmax0, unif(b0.w[0]));
            int y[kMaxM + 1] = {};
            const double* cum = lcum + (size_t)a * m;
            Block bu = b0;
            for (int i = 0; i < a; ++i) {
                if ((i & 3) == 0) bu = philox(s.seed, r, (uint64_t)t, (uint64_t)(1 + (i >> 2)));
                const double u = unif(word(bu, i & 3));
                int life = m;
                for (int k = m - 1; k >= 1; --k)
                    if (u < cum[k - 1]) life = k;
#pragma unroll
                for (int k = 1; k <= kMaxM; ++k) y[k] += life == k ? 1 : 0;
            }
            const int cap = R0 - 1;
            int before = 0, tot = 0;
#pragma unroll
            for (int j = 1; j <= kMaxM; ++j) {
                before += X[j];
                X[j] = j < m ? min(X[j] + y[j], cap) : (j == m ? y[j] : 0);
                tot += X[j];
            }
            const int z1 = X[1];
            rew = -(a > 0 ? s.cfixed : 0.0) - s.chold * posd((double)(tot - d)) -
                  s.cshort * posd((double)(d - tot)) - s.cwaste * posd((double)(z1 - d));
            int rem = d;
#pragma unroll
            for (int j = 1; j <= kMaxM; ++j) {
                const int take = min(rem, X[j]);
                X[j] -= take;
                rem -= take;
            }
            const int met = d - rem, W = X[1];
#pragma unroll
            for (int j = 1; j < kMaxM; ++j) X[j] = j < m ? X[j + 1] : 0;
            X[kMaxM] = 0;
            tau = tau + 1 == s.P ? 0 : tau + 1;
            day = Tally{d, met, W, tot - before, tot - met};
        }
        if (t >= s.warmup) {
            acc += g * rew;
            g *= s.gamma;
            add(c, day);
            if (kTwo) {
                add(c0, day0);
                add(c1, day1);
            }
        }
    }
    s.ret[lane] = acc;
    kpis(s.kpi + 3 * lane, c, s.horizon);
    if (kTwo && s.pkpi) {
        kpis(s.pkpi + 6 * lane, c0, s.horizon);
        kpis(s.pkpi + 6 * lane + 3, c1, s.horizon);
    }
}

// Mean and sample standard deviation (n - 1) of ncol columns of each policy's
// [n_roll][stride] block: one workgroup per policy, two passes, fixed summation
// order (so a column's figures do not depend on the other columns).
__global__ __launch_bounds__(256) void column_stats_kernel(const double* x, int stride, int ncol,
                                                           int n_roll, double* out, int ostride,
                                                           int ooff) {
    __shared__ double red[256];
    const int pol = blockIdx.x, tid = threadIdx.x;
    const double* xp = x + (size_t)pol * n_roll * stride;
    for (int q = 0; q < ncol; ++q) {
        double mean = 0.0;
        for (int pass = 0; pass < 2; ++pass) {
            double sum = 0.0;
            for (int i = tid; i < n_roll; i += 256) {
                const double v = xp[(size_t)i * stride + q];
                sum += pass == 0 ? v : (v - mean) * (v - mean);
            }
            red[tid] = sum;
            __syncthreads();
            for (int w = 128; w > 0; w >>= 1) {
                if (tid < w) red[tid] += red[tid + w];
                __syncthreads();
            }
            const double total = red[0];
            __syncthreads();
            if (pass == 0) {
                mean = total / (double)n_roll;
            } else if (tid == 0) {
                out[(size_t)pol * ostride + ooff + 2 * q] = mean;
                out[(size_t)pol * ostride + ooff + 2 * q + 1] =
                    n_roll > 1 ? sqrt(total / (double)(n_roll - 1)) : 0.0;
            }
        }
    }
}

hipError_t launch_rollouts(const SimDev& s, hipStream_t st) {
    const int64_t lanes = (int64_t)s.n_pol * s.n_roll;
    if (lanes <= 0) return hipSuccess;
    const int64_t blocks = (lanes + 63) / 64;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    const size_t lds = sizeof(double) * ((size_t)s.n_cdf0 + s.n_cdf1 + s.n_lcum);
    if (lds > 65536 || s.m < 1 || s.m > kMaxM || (s.family == 0 && s.L - 1 > kMaxO))
        return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)blocks), block(64);
    if (s.family == 0)
        hipLaunchKernelGGL(rollout_kernel<0>, grid, block, lds, st, s);
    else if (s.family == 1)
        hipLaunchKernelGGL(rollout_kernel<1>, grid, block, lds, st, s);
    else if (s.family == 2)
        hipLaunchKernelGGL(rollout_kernel<2>, grid, block, lds, st, s);
    else
        hipLaunchKernelGGL(rollout_kernel<3>, grid, block, lds, st, s);
    return hipGetLastError();
}

hipError_t launch_column_stats(const double* x, int stride, int ncol, int n_pol, int n_roll,
                               double* out, int ostride, int ooff, hipStream_t st) {
    if (n_pol <= 0 || n_roll <= 0 || ncol <= 0) return hipSuccess;
    if (ncol > stride || ooff + 2 * ncol > ostride) return hipErrorInvalidValue;
    hipLaunchKernelGGL(column_stats_kernel, dim3(n_pol), dim3(256), 0, st, x, stride, ncol,
                       n_roll, out, ostride, ooff);
    return hipGetLastError();
}

}  // namespace pvi
