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
//     all X_2 lie on one descending list of (m-1)(R-1)+1 points at most, and a
//     per-diagonal prefix sum over that list (kernel comment below) gives every
//     state of the tile for every action.
//
// Wavefront = G tiles (O, X_m..X_3) of one digit sum, R lanes per tile; the tile's
// path list streams through LDS.  Ties in the max go to the lowest action.  No
// atomics: every reduction is a fixed tree, so reruns are bit-identical.
#include <hip/hip_ext.h>
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

// Orders a wavefront's LDS stores before its later LDS reads of other lanes' data
// (no instruction: LDS requests of one wavefront are served in issue order).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Value staged for the padding actions R <= a < RMAX: so negative that their Q
// never wins the max, small enough that weighted sums of it (total weight <= 1)
// stay finite.  With it the action loops need no bound check.  Variants compiled
// for one exact action count (RC = R) compute no padded action at all: they stage
// the same RMAX-wide rows but keep running sums only for the R real actions, which
// frees registers and skips the padded multiply-adds; the maxima are over the same
// actions, so their results are identical.
// Elements between the staged chunks of two tiles of a wavefront: CH * RMAX, padded
// so that consecutive tiles' rows start 4 banks apart (a stride of 4 dwords modulo
// 64); the tiles' 16-byte row reads then never share a bank.
template <typename VT>
__host__ __device__ constexpr int tile_stride(int ch, int rmax) {
    const int e = ch * rmax;
    return sizeof(VT) == 8 ? e + ((2 - e) % 32 + 32) % 32 : e + ((4 - e) % 64 + 64) % 64;
}

template <typename VT>
__device__ constexpr VT kPadValue = VT(-1e30);
template <>
__device__ constexpr double kPadValue<double> = -1e300;

// One wavefront per group of G tiles of equal digit sum b; VT: storage type of V
// (float = centred FP32, double = FP64); KAHAN: FP32 compensated accumulation (only
// with VT = float), else FP64.  EXTRACT: write policy and Q gap instead of V (FP64).
//
// For a state (X_2, X_1) of a tile put N = b + X_2 (its path length) and
// u = X_1 + N.  For N >= 1,
//   E = F(X_1) S[N] + C(u, N) + G(u) S[0],   C(u, N) = sum_{j=1}^{N-1} P(u - j) S[j],
// with F = P(D <= .), G = P(D >= .) and S the tile's path list.  For a fixed u,
// C(u, N) is a running sum over the path points, walked once for every action while
// N moves up the list; the states of diagonal u (X_1 = u - N in [0, R)) are emitted
// as N passes them.  The live diagonals are u in [n0, n0 + 2R - 2], n0 = max(b, 1).
// Lane l of a tile carries two of them, u1 = n0 + l and u2 = u1 + R: at every step
// N in [n0, b + R - 1] exactly one of the two is on the emitting window
// [N, N + R - 1] (u1 while u1 >= N, then u2), so each of the R lanes emits one state
// per step and a wavefront of G = floor(64 / R) tiles keeps nearly every lane busy.
// The lane keeps A1 = C(u1) and D = C(u2) - C(u1); the emitted running sum is
// A1 + m D with m in {0, 1}, one multiply-add.  The path list streams through LDS in
// chunks of CH points, double buffered: the next chunk's values are loaded into
// registers while the current one is used.  The single-point state (N = 0, b = 0)
// takes S[0] for every demand.  All actions of a state live in one lane, so the max
// needs no exchange.  Weights are staged premultiplied by gamma.
template <typename VT, bool KAHAN, int RMAX, bool EXTRACT, int RC>
__device__ __forceinline__ void backup_a_body(ADev p, unsigned char* smem) {
    Ctl* ctl = p.ctl;
    if (!EXTRACT && ctl->stop) return;
    constexpr int W = VecLoad<VT>::W;
    constexpr int SPL = 8;              // actions one staging lane loads
    constexpr int NSPLIT = RMAX / SPL;  // staging lanes per path point
    using VV = typename VecLoad<VT>::V;
    using AW = typename Acc<VT, KAHAN>::W;

    const int R = p.R, m = p.m, G = p.G, CH = p.CH, lane = threadIdx.x;
    const int grp = xcd_remap(blockIdx.x, gridDim.x);
    const int32_t* gt = p.groups + (size_t)grp * G;
    const int first = gt[0];  // a group's first slot always holds a tile

    // compute role: tile slot g, position l.  Lanes past G * R and the slots of a
    // short group repeat a lane of tile `first`: they compute and store exactly that
    // lane's values, so every lane loads and stores unconditionally (which also
    // lets the compiler count outstanding memory operations exactly).
    int g = lane / R;
    const int l = lane - g * R;
    if (g >= G) g = 0;
    int tile = gt[g];
    if (tile < 0) tile = first;
    // digit sum of the group's tiles (equal for all of them), taken from the first
    // so that it and the loop bounds are wavefront-uniform
    int b = 0;
    {
        int t = first % p.nz;
        for (int i = 2; i <= m - 1; ++i) {
            b += t % R;
            t /= R;
        }
    }
    const int lp = b + p.r2;  // path points 0 .. lp - 1
    const int lpm = (m >= 2 ? (m - 2) * (R - 1) : 0) + p.r2;  // longest path list

    // staging role: action slice sh, tile slot sg, point sj of every chunk; lanes
    // past the stagers repeat the first stager's loads and store nothing
    const int npair = G * CH;
    const bool stager = lane < NSPLIT * npair;
    const int sl = stager ? lane : 0;
    const int sh = sl / npair, spair = sl - sh * npair;
    const int sg = spair / CH, sj = spair - sg * CH;
    int64_t s_base = 0;
    {
        int st = gt[sg];
        if (st < 0) st = first;
        s_base = (int64_t)(st / p.nz) * p.stride_h;
    }

    // [2][G][TS] with TS >= CH * RMAX: chunk c & 1, tile slot, point-major rows of RMAX
    const int TS = tile_stride<VT>(CH, RMAX);
    VT* buf = reinterpret_cast<VT*>(smem);
    // RMAX and TS are multiples of 2 doubles or 4 floats, so every staged row starts on
    // a 16-byte boundary
    // weight tables (premultiplied by gamma): F and G indexed by d; and, walked upwards
    // as N grows, the reversed tables Pr[j] = P(k) and Dr[j] = P(k + R) - P(k) at
    // k = tab - 1 - j, with P(k) read as 0 for k <= 0 and k >= tab (d = 0 never enters
    // a running sum, and the PMF is zero beyond d_max): a lane's weights at point N are
    // Pr and Dr at (tab - 1 - u1) + N, with no bound checks
    const int TW = p.tab + R;
    double* sF = reinterpret_cast<double*>(smem + sizeof(VT) * (size_t)2 * G * TS);
    double* sG = sF + p.tab;
    double* sPr = sG + p.tab;
    double* sDr = sPr + TW;
    int* soff = reinterpret_cast<int*>(sDr + TW);  // [G][lpm] block offset of each point
    const VT* vin = reinterpret_cast<const VT*>(p.v_in);

    const double gm = p.gamma;
    for (int i = lane; i < p.tab; i += 64) {
        sF[i] = gm * p.cdf[i];
        sG[i] = gm * p.tail[i];
    }
    for (int j = lane; j < TW; j += 64) {
        const int k = p.tab - 1 - j, k2 = k + R;
        const double pk = k >= 1 ? gm * p.pmf[k] : 0.0;
        const double pk2 = (k2 >= 1 && k2 < p.tab) ? gm * p.pmf[k2] : 0.0;
        sPr[j] = pk;
        sDr[j] = pk2 - pk;
    }
    for (int i = lane; i < G * lp; i += 64) {
        const int gg = i / lp, j = i - gg * lp;
        int st = gt[gg];
        if (st < 0) st = first;
        int t = st % p.nz, Y[9];
        for (int k = 2; k <= m - 1; ++k) {
            Y[k] = t % R;
            t /= R;
        }
        soff[gg * lpm + j] = path_offset(j, Y, m, p.pow_y);
    }
    wave_sync();

    VT pre[SPL];
    auto load_chunk = [&](int c) {
        const int j = min(c * CH + sj, lp - 1);
        const VT* src = vin + s_base + soff[sg * lpm + j];
        // raw loads only: the padding is applied when the chunk is stored, so the
        // loads stay in flight until then
#pragma unroll
        for (int e = 0; e < SPL; ++e) pre[e] = src[(int64_t)min(sh * SPL + e, R - 1) * p.stride_a];
    };
    auto store_chunk = [&](int c) {
        if (stager && c * CH + sj < lp) {
            VV* dst = reinterpret_cast<VV*>(buf + (size_t)((c & 1) * G + sg) * TS + sj * RMAX +
                                            sh * SPL);
            VT v[SPL];
#pragma unroll
            for (int e = 0; e < SPL; ++e) v[e] = sh * SPL + e < R ? pre[e] : kPadValue<VT>;
#pragma unroll
            for (int q = 0; q < SPL / W; ++q) dst[q] = make_vec<VT>(&v[q * W]);
        }
    };

    load_chunk(0);
    store_chunk(0);
    wave_sync();
    const int nchunks = (lp + CH - 1) / CH;
    if (nchunks > 1) load_chunk(1);

    const int ns_tile = p.r2 * R;
    const int64_t tbase = (int64_t)tile * ns_tile;
    const double mu = (!EXTRACT && sizeof(VT) == 4) ? ctl->mu : 0.0;
    const double cv = p.cvar;
    double dmx = -DBL_MAX, dmn = DBL_MAX, vmx = -DBL_MAX, vmn = DBL_MAX;

    // r0n and vold are the state's reward-table entry and its current value,
    // loaded ahead of time by the caller
    auto finish = [&](uint32_t s_idx, double best, double second, int arg, double r0n,
                      double vold) {
        if (EXTRACT) {
            p.pi[s_idx] = arg;
            p.gap[s_idx] = R > 1 ? best - second : INFINITY;
        } else {
            const VT o = (VT)(r0n - mu + best);
            reinterpret_cast<VT*>(p.v_out)[s_idx] = o;
            const double out = (double)o, dv = out - vold;
            dmx = fmax(dmx, dv);
            dmn = fmin(dmn, dv);
            if constexpr (sizeof(VT) == 4) {  // the FP32 centring needs the value range
                vmx = fmax(vmx, out);
                vmn = fmin(vmn, out);
            }
        }
    };
    auto take = [&](double qv, int a, double& best, double& second, int& arg) {
        if (qv > best) {
            second = best;
            best = qv;
            arg = a;
        } else if (qv > second) {
            second = qv;
        }
    };

    const VV* row0 = reinterpret_cast<const VV*>(buf + (size_t)g * TS);
    // N = 0 (only when b = 0): nothing left to deplete, every demand lands on S[0]
    if (b == 0) {
        double r0n = 0.0, vold = 0.0;
        if (!EXTRACT) {
            r0n = p.r0[l * p.xt + l];
            vold = (double)vin[tbase + l];
        }
        double best = -DBL_MAX, second = -DBL_MAX;
        int arg = 0;
#pragma unroll
        for (int q = 0; q < (RC + W - 1) / W; ++q) {
            const VV s0 = row0[q];
#pragma unroll
            for (int e = 0; e < W; ++e) {
                const int a = q * W + e;
                if (a >= RC) break;
                const double qv = fma(gm, (double)lane_of<VT, W>(s0, e), -cv * a);
                if (EXTRACT)
                    take(qv, a, best, second, arg);
                else
                    best = fmax(best, qv);
            }
        }
        finish((uint32_t)tbase + l, best, second, arg, r0n, vold);
    }

    const int n0 = b > 1 ? b : 1, nmax = lp - 1;
    const int u1 = n0 + l, u2 = u1 + R;
    // start from the j = 0 term G(u) S[0] (and, with FP64 accumulation, the order
    // cost, which the difference D does not carry)
    Acc<VT, KAHAN> A1[RC], D[RC];
    {
        const double g1 = sG[u1], g2 = sG[u2];
        const AW gd = (AW)(g2 - g1);
#pragma unroll
        for (int q = 0; q < (RC + W - 1) / W; ++q) {
            const VV s0 = row0[q];
#pragma unroll
            for (int e = 0; e < W; ++e) {
                const int a = q * W + e;
                if (a >= RC) break;
                const VT sv = lane_of<VT, W>(s0, e);
                if constexpr (KAHAN)
                    A1[a].add((AW)g1, sv);
                else
                    A1[a].s = fma(g1, (double)sv, -cv * a);
                D[a].add(gd, sv);
            }
        }
    }

    int c = 0, cj = 0;  // chunk of the current point and position inside it
    // moves to the next point; on entering chunk c + 1 publishes it and starts
    // loading chunk c + 2
    auto advance = [&]() {
        if (++cj == CH) {
            cj = 0;
            ++c;
            store_chunk(c);
            // the workgroup is this one wavefront, whose LDS operations run in
            // issue order: only the compiler has to keep the stores before the reads
            wave_sync();
            if (c + 1 < nchunks) load_chunk(c + 1);
        }
    };
    auto point = [&]() {
        return reinterpret_cast<const VV*>(buf + (size_t)((c & 1) * G + g) * TS + cj * RMAX);
    };
    // weights of point N for the two running sums, P(u1 - N) and P(u2 - N) - P(u1 - N)
    // (a diagonal with u - N <= 0 is finished and adds nothing)
    const int wbase = p.tab - 1 - u1;
    auto weights = [&](int N, AW& w1, AW& wd) {
        w1 = (AW)sPr[wbase + N];
        wd = (AW)sDr[wbase + N];
    };

    // points 1 .. n0 - 1 precede every state of the group: running sums only
    for (int N = 1; N < n0; ++N) {
        advance();
        const VV* rN = point();
        AW w1, wd;
        weights(N, w1, wd);
#pragma unroll
        for (int q = 0; q < (RC + W - 1) / W; ++q) {
            const VV sq = rN[q];
#pragma unroll
            for (int e = 0; e < W; ++e) {
                if (q * W + e >= RC) break;
                const VT svt = lane_of<VT, W>(sq, e);
                A1[q * W + e].add(w1, svt);
                D[q * W + e].add(wd, svt);
            }
        }
    }

    // The state a lane emits at point N >= n0 has X_2 = N - b and X_1 = u1 - N while
    // N <= u1, then u2 - N: X_1 steps down by one and wraps once, from 0 to R - 1.  Its
    // index tbase + X_2 R + X_1 then grows by R - 1, or 2R - 1 at the wrap, and its
    // reward-table index X_1 (xt + 1) + N by 1 - (xt + 1) or 1 + (R - 1)(xt + 1).  The
    // reward entry and old value of the state PD points ahead are loaded into one of
    // PD register slots (the loop is unrolled by PD, so each slot is used and then
    // refilled in place, with no register move that would force the load to complete
    // early); past the last point the loads read the tile's first state instead.
    constexpr int PD = 3;
    struct Walk {
        int x;         // X_1
        uint32_t s;    // state index
        uint32_t r;    // reward-table index
    };
    const int xt1 = p.xt + 1;
    // next point: the wrap adds R to X_1 (unsigned minimum of x - 1 and x - 1 + R)
    auto step_walk = [&](Walk& w) {
        const uint32_t t = (uint32_t)(w.x - 1), tw = (uint32_t)(w.x - 1 + R);
        const uint32_t x = min(t, tw);
        const uint32_t d = x - t;  // R at the wrap, else 0
        w.x = (int)x;
        w.s += (uint32_t)(R - 1) + d;
        w.r = w.r + 1u - (uint32_t)xt1 + d * (uint32_t)xt1;
    };
    const uint32_t tb = (uint32_t)tbase;
    Walk cur{l, tb + (uint32_t)((n0 - b) * R + l), (uint32_t)(l * xt1 + n0)};
    Walk ahd = cur;
    auto prefetch = [&](int N, double& r0s, double& vs) {
        if constexpr (!EXTRACT) {
            const bool live = N <= nmax;  // the same for every lane
            r0s = p.r0[live ? ahd.r : 0u];
            vs = (double)vin[live ? ahd.s : tb];
            step_walk(ahd);
        }
    };

    // points n0 .. nmax: every lane emits one state per point.  Each pair (or
    // quad) of actions of the point is read, used for the state and both sums,
    // and dropped, so the row is never held whole.  The sums are also advanced
    // after the last point (unused), which keeps the body free of branches.
    auto step = [&](int N, double& r0s, double& vs) {
        advance();
        const VV* rN = point();
        AW w1, wd;
        weights(N, w1, wd);
        const double fwr = sF[min(cur.x, p.dmax)];
        // Q_a = gamma (F(X_1) S[N][a] + C(u, N) + G(u) S[0][a]) - c_var a, with
        // C(u, N) = A1 + D once the lane is on its second diagonal
        const double msel = u1 < N ? 1.0 : 0.0;
        double best = -DBL_MAX, second = -DBL_MAX;
        int arg = 0;
        double bq[4];
#pragma unroll
        for (int q = 0; q < (RC + W - 1) / W; ++q) {
            const VV sq = rN[q];
#pragma unroll
            for (int e = 0; e < W; ++e) {
                const int a = q * W + e;
                if (a >= RC) break;
                const VT svt = lane_of<VT, W>(sq, e);
                const double sv = (double)svt;
                const double run = fma(msel, D[a].value(), A1[a].value());
                if constexpr (EXTRACT) {
                    take(fma(fwr, sv, run), a, best, second, arg);
                } else {
                    const double qv = KAHAN ? fma(fwr, sv, run) - cv * a : fma(fwr, sv, run);
                    bq[a & 3] = a < 4 ? qv : fmax(bq[a & 3], qv);
                }
                A1[a].add(w1, svt);
                D[a].add(wd, svt);
            }
        }
        if (!EXTRACT) {
            static_assert(RC >= 4, "the partial maxima need four actions");
            best = fmax(fmax(bq[0], bq[1]), fmax(bq[2], bq[3]));
        }
        finish(cur.s, best, second, arg, r0s, vs);
        step_walk(cur);
        prefetch(N + PD, r0s, vs);  // the slot is consumed: refill it for step N + PD
    };
    double ra = 0.0, va = 0.0, rb = 0.0, vb = 0.0, rc = 0.0, vc = 0.0;
    prefetch(n0, ra, va);
    prefetch(n0 + 1, rb, vb);
    prefetch(n0 + 2, rc, vc);
    for (int N = n0; N <= nmax; N += PD) {
        step(N, ra, va);
        if (N + 1 > nmax) break;
        step(N + 1, rb, vb);
        if (N + 2 > nmax) break;
        step(N + 2, rc, vc);
    }
    if (EXTRACT) return;
    dmx = wave_max(dmx);
    dmn = wave_min(dmn);
    vmx = wave_max(vmx);
    vmn = wave_min(vmn);
    if (lane == 0) {
        double* pp = p.partials + 4 * (size_t)grp;
        pp[0] = dmx;
        pp[1] = dmn;
        pp[2] = vmx;
        pp[3] = vmn;
    }
}

// Two entry points of one body: the first asks for two wavefronts per SIMD (its
// registers fit in 256), the second has the whole register file for the variants
// that would spill at that budget (RMAX = 32, FP32 compensated sums at RMAX >= 16).
template <typename VT, bool KAHAN, int RMAX, bool EXTRACT, int RC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void
backup_a_kernel(ADev p) {
    extern __shared__ __align__(16) unsigned char smem[];
    backup_a_body<VT, KAHAN, RMAX, EXTRACT, RC>(p, smem);
}

template <typename VT, bool KAHAN, int RMAX, bool EXTRACT, int RC>
__global__ __launch_bounds__(64) void backup_a_wide_kernel(ADev p) {
    extern __shared__ __align__(16) unsigned char smem[];
    backup_a_body<VT, KAHAN, RMAX, EXTRACT, RC>(p, smem);
}

// Single-workgroup reduction of the per-tile partials and the stopping rule.
__global__ __launch_bounds__(1024) void span_kernel(Ctl* ctl, const double* partials,
                                                    int tiles, int fp32, int fixed,
                                                    double gamma) {
    __shared__ double red[4 * 16];
    // the control block and up to four partials per thread are requested together,
    // so the reduction waits for one memory round trip (partials are always
    // readable; after the stop flag they are simply not used)
    const Ctl cur = *ctl;
    double a0 = -DBL_MAX, a1 = DBL_MAX, a2 = -DBL_MAX, a3 = DBL_MAX;
    const double2* pp = reinterpret_cast<const double2*>(partials);
    const int bd = blockDim.x;
    int i = threadIdx.x;
    auto take = [&](double2 x, double2 y) {
        a0 = fmax(a0, x.x);
        a1 = fmin(a1, x.y);
        a2 = fmax(a2, y.x);
        a3 = fmin(a3, y.y);
    };
    // four loads per round, past the end repeating the last partial (max and min
    // are unchanged by a repeat)
    for (; i < tiles; i += 4 * bd) {
        double2 x[4], y[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int t = min(i + k * bd, tiles - 1);
            x[k] = pp[2 * t];
            y[k] = pp[2 * t + 1];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) take(x[k], y[k]);
    }
    if (cur.stop) return;
    block_reduce4(a0, a1, a2, a3, red);
    if (threadIdx.x != 0) return;
    Ctl next = cur;
    span_update(next, a0, a1, a2, a3, fp32, fixed, gamma);
    *ctl = next;
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

template <typename VT, bool KAHAN, bool EXTRACT, int RMAX, int RC = RMAX>
static hipError_t launch_a_r(const ADev& p, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    const int lp_max = (p.m >= 2 ? (p.m - 2) * (p.R - 1) : 0) + p.r2;
    // lanes: G tiles of R lanes; staging: RMAX / 8 action slices of G x CH points
    if (p.G < 1 || p.G * p.R > 64 || p.CH < 1 || (RMAX / 8) * p.G * p.CH > 64 ||
        p.ngroups < 1)
        return hipErrorInvalidConfiguration;
    size_t bytes = sizeof(VT) * (size_t)2 * p.G * tile_stride<VT>(p.CH, RMAX);
    bytes += sizeof(double) * (2 * (size_t)p.tab + 2 * ((size_t)p.tab + p.R)) +
             sizeof(int) * (size_t)p.G * lp_max;
    if (bytes > 65536) return hipErrorInvalidConfiguration;
    // G is read at u2 <= b + 2R and P, F at clamped indices
    if (p.tab < 2 * p.R + lp_max + 1 || p.tab < p.dmax + 2) return hipErrorInvalidValue;
    constexpr bool wide = RMAX == 32 || (KAHAN && RMAX >= 16);
    // with events, they are recorded by the launch itself at the kernel's start and end
    if constexpr (wide) {
        if (ev0 || ev1)
            hipExtLaunchKernelGGL((backup_a_wide_kernel<VT, KAHAN, RMAX, EXTRACT, RC>),
                                  dim3(p.ngroups), dim3(64), (uint32_t)bytes, s, ev0, ev1, 0, p);
        else
            hipLaunchKernelGGL((backup_a_wide_kernel<VT, KAHAN, RMAX, EXTRACT, RC>),
                               dim3(p.ngroups), dim3(64), bytes, s, p);
    } else {
        if (ev0 || ev1)
            hipExtLaunchKernelGGL((backup_a_kernel<VT, KAHAN, RMAX, EXTRACT, RC>), dim3(p.ngroups),
                                  dim3(64), (uint32_t)bytes, s, ev0, ev1, 0, p);
        else
            hipLaunchKernelGGL((backup_a_kernel<VT, KAHAN, RMAX, EXTRACT, RC>), dim3(p.ngroups),
                               dim3(64), bytes, s, p);
    }
    return hipGetLastError();
}

template <typename VT, bool KAHAN, bool EXTRACT>
static hipError_t launch_a_t(const ADev& p, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    // exact action counts of the paper's scenario A (order cap 10) and of the
    // order cap 20 instances; at R = 11 the FP64 variant fits three wavefronts per SIMD
    if (p.R == 11) return launch_a_r<VT, KAHAN, EXTRACT, 16, 11>(p, s, ev0, ev1);
    if (p.R == 21) return launch_a_r<VT, KAHAN, EXTRACT, 24, 21>(p, s, ev0, ev1);
    if (p.R <= 8) return launch_a_r<VT, KAHAN, EXTRACT, 8>(p, s, ev0, ev1);
    if (p.R <= 16) return launch_a_r<VT, KAHAN, EXTRACT, 16>(p, s, ev0, ev1);
    if (p.R <= 24) return launch_a_r<VT, KAHAN, EXTRACT, 24>(p, s, ev0, ev1);
    if (p.R <= 32) return launch_a_r<VT, KAHAN, EXTRACT, 32>(p, s, ev0, ev1);
    return hipErrorInvalidValue;
}

hipError_t launch_backup_a(const ADev& p, int storage_fp32, int acc_kahan, int extract,
                           hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (extract) return launch_a_t<double, false, true>(p, s, ev0, ev1);
    if (storage_fp32) {
        if (acc_kahan) return launch_a_t<float, true, false>(p, s, ev0, ev1);
        return launch_a_t<float, false, false>(p, s, ev0, ev1);
    }
    return launch_a_t<double, false, false>(p, s, ev0, ev1);
}

hipError_t launch_span(Ctl* ctl, const double* partials, int tiles, int storage_fp32,
                       int fixed, double gamma, hipStream_t s) {
    // a block no wider than the partials need (whole wavefronts, at most 1024): small
    // instances then pay for one wavefront, not sixteen; max and min are exact, so
    // the block width does not change the result
    const int threads = tiles >= 1024 ? 1024 : tiles <= 64 ? 64 : (tiles + 63) / 64 * 64;
    hipLaunchKernelGGL(span_kernel, dim3(1), dim3(threads), 0, s, ctl, partials, tiles,
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
