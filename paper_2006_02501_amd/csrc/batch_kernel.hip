// Batched form: thousands of independent small systems (1..64 bodies each)
// advanced for many P(EC)^n steps in ONE persistent kernel launch.
//
// Systems are packed first-fit-decreasing into 64-lane bins on the host (one
// lane per body).  Each workgroup is a single wave64; it takes the next bin
// from a device counter (bins are ordered longest first), keeps every body's
// state (x, v, a^(0..2p-1)) in VGPRs for all steps, and exchanges the
// predicted / corrected path of the current iterate through LDS.  The only
// global traffic per bin is the initial load, the final store and one counter
// increment.  An evaluation takes each pair of a system once, for both of its
// bodies, in a sweep over the bin's lanes (see the kernel); an idle lane, or a
// lane without a pair in a sweep step, contributes zero.  Systems may take
// different iteration counts n: a bin iterates as often as its largest n, and
// a system stops correcting (and keeps its last iterate) after its own.
#include "hermite_coeffs.h"
#include "kernels.h"
#include "lane_moves.h"
#include "pair_chain.h"

namespace hermite {
namespace {

constexpr int kLanes = 64;

struct LaneInfo {
    int sys;       // system of this lane (-1: idle lane)
    int lo, hi;    // slot range of that system inside the bin
    int maxlen;    // largest system in the bin
    int64_t g;     // global particle index
    int maxiter;   // largest iteration count in the bin (with per-system counts)
};

__device__ __forceinline__ LaneInfo lane_info(const BatchPlan &pl, int b, int lane, const int *iters = nullptr)
{
    LaneInfo li{-1, lane, lane + 1, 0, 0, 0};
    const int s0 = pl.bin_start[b], s1 = pl.bin_start[b + 1];
    int base = 0;
    for (int k = s0; k < s1; ++k) {
        const int s = pl.bin_sys[k];
        const int64_t off = pl.offsets[s];
        const int sz = (int)(pl.offsets[s + 1] - off);
        li.maxlen = max(li.maxlen, sz);
        if (iters) li.maxiter = max(li.maxiter, iters[s]);
        if (lane >= base && lane < base + sz) {
            li.sys = s;
            li.lo = base;
            li.hi = base + sz;
            li.g = off + (lane - base);
        }
        base += sz;
    }
    return li;
}

struct Path6 {
    const double *p[6];
};

// One generic-order initialisation pass for every system of bin blockIdx.x.
template <int K>
__global__ __launch_bounds__(kLanes) void batch_init_kernel(BatchPlan pl, int64_t n, const double *__restrict__ mass,
                                                            Path6 path, int k_first, double G, double eps2,
                                                            double *__restrict__ out)
{
    __shared__ double sm[kLanes];
    __shared__ double sp[K + 1][3][kLanes];
    const int lane = threadIdx.x;
    const LaneInfo li = lane_info(pl, blockIdx.x, lane);
    const bool active = li.sys >= 0;
    sm[lane] = active ? G * mass[li.g] : 0.0;
#pragma unroll
    for (int k = 0; k <= K; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) sp[k][c][lane] = active ? path.p[k][c * n + li.g] : 0.0;
    __syncthreads();
    double xi[K + 1][3], acc[K + 1][3];
#pragma unroll
    for (int k = 0; k <= K; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xi[k][c] = sp[k][c][lane];
            acc[k][c] = 0.0;
        }
    for (int t = 0; t < li.maxlen; ++t) {
        const int j = li.lo + t;
        const bool act = active && j < li.hi && j != lane;
        const int jc = act ? j : lane;
        double r[K + 1][3];
#pragma unroll
        for (int k = 0; k <= K; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) r[k][c] = sp[k][c][jc] - xi[k][c];
        generic_accumulate<K>(r, eps2, sm[jc], !act, acc);
    }
    if (!active) return;
#pragma unroll
    for (int k = 0; k <= K; ++k) {
        if (k < k_first) continue;
#pragma unroll
        for (int c = 0; c < 3; ++c) out[((int64_t)(k - k_first) * 3 + c) * n + li.g] = acc[k][c];
    }
}

// Bins whose largest system has at least this many bodies sweep the whole
// wave as one ring: 32 steps, sums moved by DPP.  The others sweep each system
// as a ring of its own: largest/2 steps, sums moved by permutes, which go
// through the LDS unit and make a step about a third dearer with two waves
// per SIMD.  Measured on the 4096-system workload: 57 and 61 best, 49 ~1 %
// and 41 ~5 % slower, no ring at all ~3 % (FP64) and ~10 % (mixed) slower.
constexpr int kRingMin = 57;

__global__ void reset_counter_kernel(int *counter) { counter[0] = 0; }

__device__ constexpr double kInvB[9] = {0.0, 1.0, 1.0 / 2.0, 1.0 / 3.0, 1.0 / 4.0, 1.0 / 5.0, 1.0 / 6.0, 1.0 / 7.0, 1.0 / 8.0};

template <int P, bool MIXED, int CORR, bool COMP>
__global__ __launch_bounds__(kLanes) void batch_run_kernel(BatchPlan pl, int64_t n, const double *__restrict__ mass,
                                                           double *__restrict__ pos, double *__restrict__ vel,
                                                           double *__restrict__ deriv,
                                                           const double *__restrict__ dt_sys, int n_steps,
                                                           int n_iter, const int *__restrict__ iters, double G,
                                                           double eps2, double *__restrict__ comp)
{
    constexpr int K = P;
    // chain arithmetic: FP64, or FP32 from the FP64 differences (mixed)
    using T = typename std::conditional<MIXED, float, double>::type;
    // two sweep steps in flight; the 8th-order FP64 kernel with compensation
    // would exceed 256 registers with them
    constexpr bool kTwoSteps = !(P == 3 && !MIXED && COMP);
    __shared__ T sgm[kLanes];
    __shared__ double sp[K + 1][3][kLanes];
    __shared__ double wait_xv[COMP ? 12 : 1][kLanes];
    __shared__ int next_bin;
    const int lane = threadIdx.x;
    const int64_t n3 = 3 * n;

    for (;;) {
        if (lane == 0) next_bin = atomicAdd(pl.counter, 1);
        __syncthreads();
        const int b = next_bin;
        __syncthreads();
        if (b >= pl.n_bins) break;
        const LaneInfo li = lane_info(pl, b, lane, iters);
        const bool active = li.sys >= 0;
        // iterations of this bin and of this lane's system (the host checks
        // every count is in 1..64)
        const int bin_iter = iters ? li.maxiter : n_iter;
        const int my_iter = (iters && active) ? iters[li.sys] : bin_iter;

        double x[3], v[3], d[2 * P][3];
        // Kahan compensation of x and v (COMP, the option of Sec. 3.2):
        // the carried terms, and the ones the latest correction produced
        double cx[3] = {0.0, 0.0, 0.0}, cv[3] = {0.0, 0.0, 0.0};
        double ncx[3] = {0.0, 0.0, 0.0}, ncv[3] = {0.0, 0.0, 0.0};
        double dt = 1.0;
        if (active) {
            dt = dt_sys[li.sys];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                x[c] = pos[c * n + li.g];
                v[c] = vel[c * n + li.g];
                if constexpr (COMP) {
                    cx[c] = comp[c * n + li.g];
                    cv[c] = comp[n3 + c * n + li.g];
                }
#pragma unroll
                for (int k = 0; k < 2 * P; ++k) d[k][c] = deriv[k * n3 + c * n + li.g];
            }
        } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                x[c] = 1.0e3 * (lane + 1);   // far from every real body; contributes nothing (mass 0)
                v[c] = 0.0;
#pragma unroll
                for (int k = 0; k < 2 * P; ++k) d[k][c] = 0.0;
            }
        }
        const double gm = active ? G * mass[li.g] : 0.0;
        const T gm_own = (T)gm;
        sgm[lane] = gm_own;
        // The bin's sweep (every pair of each system once, see below): its
        // kind, its step count, the lane a segment sweep passes sums from, and
        // the lane holding this body's j-side sums after the sweep.
        const int sz = li.hi - li.lo, q = lane - li.lo, half = sz / 2;
        const bool ring = li.maxlen >= kRingMin;
        const int nsweep = ring ? min(li.maxlen - 1, kLanes / 2) : li.maxlen / 2;
        const int succ = 4 * (li.lo + (q + 1 == sz ? 0 : q + 1));
        int hq = q - nsweep % sz;
        hq = hq < 0 ? hq + sz : hq;
        const int home = 4 * (ring ? ((lane - nsweep) & (kLanes - 1)) : li.lo + hq);

        for (int step = 0; step < n_steps; ++step) {
            // Taylor predictor from the t0 state (Horner form).
            double path[K + 1][3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double xs[2 * P + 2];
                xs[0] = x[c];
                xs[1] = v[c];
#pragma unroll
                for (int k = 0; k < 2 * P; ++k) xs[k + 2] = d[k][c];
#pragma unroll
                for (int f = 0; f <= K; ++f) {
                    const int M = 2 * P + 1 - f;
                    double s = xs[f + M];
#pragma unroll
                    for (int k = M - 1; k >= 0; --k) s = __builtin_fma(s, dt * kInvB[k + 1], xs[f + k]);
                    path[f][c] = s;
                }
            }
            double a1[K + 1][3];
            double x1[3], v1[3];
            for (int it = 0; it < bin_iter; ++it) {
                __syncthreads();
#pragma unroll
                for (int k = 0; k <= K; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) sp[k][c][lane] = path[k][c];
                __syncthreads();
                // Evaluate a^(0..P) over the lane's own system, every pair
                // once: the pair's chain adds to this lane's sums (the i-side)
                // and, with the opposite sign and the other mass, to sums that
                // travel with the partner (the j-side), passed one lane on
                // between steps; after the sweep they go back to their body.
                //  - ring: the whole wave is one ring; in step t = 1..nsweep
                //    lane l takes lane l + t (mod 64) if it is of the same
                //    system (at t = 32 only from lanes 0..31).  A system is
                //    contiguous, so each of its pairs is at ring distance
                //    <= min(maxlen - 1, 32) one way round.
                //  - segments: each system is a ring of its own; in step
                //    t = 1..sz/2 local body q takes q + t (mod sz) (at t = sz/2
                //    of an even sz only from its first half).
                T acc[K + 1][3], accj[K + 1][3];
#pragma unroll
                for (int k = 0; k <= K; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        acc[k][c] = T(0);
                        accj[k][c] = T(0);
                    }
                // the sweep, RING a compile-time tag (one loop per kind)
                auto sweep = [&](auto ring_tag) {
                    constexpr bool RING = decltype(ring_tag)::value;
                    auto step = [&](int t) {
                        int jc;
                        bool act;
                        if constexpr (RING) {
                            const int pl = (lane + t) & (kLanes - 1);
                            act = pl >= li.lo && pl < li.hi && !(t == kLanes / 2 && lane >= kLanes / 2);
                            jc = pl;
                        } else {
                            int q2 = q + t;
                            q2 = q2 >= sz ? q2 - sz : q2;
                            act = t <= half && !(2 * t == sz && q >= half);
                            jc = li.lo + q2;
                        }
                        jc = act ? jc : lane;   // no pair: zero differences, zero weight
                        T r[3], vv[3], aa[3], jj[3];
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            r[c] = (T)(sp[0][c][jc] - path[0][c]);
                            vv[c] = (T)(sp[1][c][jc] - path[1][c]);
                            aa[c] = K >= 2 ? (T)(sp[K >= 2 ? 2 : 0][c][jc] - path[K >= 2 ? 2 : 0][c]) : T(0);
                            jj[c] = K >= 3 ? (T)(sp[K >= 3 ? 3 : 0][c][jc] - path[K >= 3 ? 3 : 0][c]) : T(0);
                        }
                        T w = fma_t(r[0], r[0], fma_t(r[1], r[1], fma_t(r[2], r[2], (T)eps2)));
                        w = act ? w : T(1);
                        const T rinv = rsqrt_t(w);
                        const T rinv2 = rinv * rinv;
                        const T q3 = act ? rinv * rinv2 : T(0);
                        chain_pair<K, T>(r, vv, aa, jj, sgm[jc] * q3, -gm_own * q3, rinv2, acc, accj);
                    };
                    auto pass_on = [&]() {
#pragma unroll
                        for (int k = 0; k <= K; ++k)
#pragma unroll
                            for (int c = 0; c < 3; ++c) {
                                if constexpr (RING) accj[k][c] = lane_down(accj[k][c]);
                                else accj[k][c] = lane_from(succ, accj[k][c]);
                            }
                    };
                    int t = 1;
                    if (nsweep >= 1) {
                        step(1);
                        t = 2;
                    }
                    if constexpr (kTwoSteps) {
                        for (; t + 1 <= nsweep; t += 2) {
                            pass_on();
                            step(t);
                            pass_on();
                            step(t + 1);
                        }
                    }
                    for (; t <= nsweep; ++t) {
                        pass_on();
                        step(t);
                    }
                };
                if (ring) sweep(std::true_type{});
                else sweep(std::false_type{});
                // lane l now holds the j-side sums of body l + nsweep (ring) or
                // of local body q + nsweep (segments)
#pragma unroll
                for (int k = 0; k <= K; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) accj[k][c] = lane_from(home, accj[k][c]);
                // a system past its own iteration count keeps its last iterate
                if (it >= my_iter) continue;
#pragma unroll
                for (int k = 0; k <= K; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) a1[k][c] = (double)acc[k][c] + (double)accj[k][c];
                // Modified corrector: velocity first, then position.
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    double dv = 0.0;
#pragma unroll
                    for (int k = P; k >= 0; --k) {
                        const double s = (k & 1) ? (a1[k][c] - d[k][c]) : (a1[k][c] + d[k][c]);
                        dv = __builtin_fma(dv, dt, CV[P][k] * s);
                    }
                    if constexpr (COMP) {
                        const double y = dv * dt - cv[c];
                        v1[c] = v[c] + y;
                        ncv[c] = (v1[c] - v[c]) - y;
                    } else {
                        v1[c] = __builtin_fma(dv, dt, v[c]);
                    }
                    double dx = 0.0;
#pragma unroll
                    for (int k = P + 1; k >= 1; --k) {
                        const double s = (k & 1) ? (a1[k - 1][c] - d[k - 1][c]) : (a1[k - 1][c] + d[k - 1][c]);
                        dx = __builtin_fma(dx, dt, CX[CORR][P][k] * s);
                    }
                    dx = __builtin_fma(dx, dt, CX[CORR][P][0] * (v1[c] + v[c]));
                    if constexpr (COMP) {
                        const double y = dx * dt - cx[c];
                        x1[c] = x[c] + y;
                        ncx[c] = (x1[c] - x[c]) - y;
                    } else {
                        x1[c] = __builtin_fma(dx, dt, x[c]);
                    }
                }
                if (it + 1 < my_iter) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        path[0][c] = x1[c];
                        path[1][c] = v1[c];
#pragma unroll
                        for (int m = 0; m <= K - 2; ++m) path[2 + m][c] = a1[m][c];
                    }
                }
                if constexpr (COMP) {
                    // with compensation the iterate's x, v and their new
                    // compensation terms wait in LDS (this lane's slots) over
                    // later iterations: registers stay within 256
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        wait_xv[c][lane] = x1[c];
                        wait_xv[3 + c][lane] = v1[c];
                        wait_xv[6 + c][lane] = ncx[c];
                        wait_xv[9 + c][lane] = ncv[c];
                    }
                }
            }
            if constexpr (COMP) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    x1[c] = wait_xv[c][lane];
                    v1[c] = wait_xv[3 + c][lane];
                    ncx[c] = wait_xv[6 + c][lane];
                    ncv[c] = wait_xv[9 + c][lane];
                }
            }
            // End of step: interpolated higher derivatives, then the new state.
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if constexpr (P == 2) {
                    const double num = I6_A0[0] * d[0][c] + I6_A1[0] * a1[0][c] +
                                       (I6_A0[1] * d[1][c] + I6_A1[1] * a1[1][c]) * dt +
                                       (I6_A0[2] * d[2][c] + I6_A1[2] * a1[2][c]) * (dt * dt);
                    d[3][c] = num / (dt * dt * dt);
                }
                if constexpr (P == 3) {
                    const double tp[4] = {1.0, dt, dt * dt, dt * dt * dt};
                    double n4 = 0.0, n5 = 0.0;
#pragma unroll
                    for (int m = 0; m <= 3; ++m) {
                        n4 += (I8_4_A0[m] * d[m][c] + I8_4_A1[m] * a1[m][c]) * tp[m];
                        n5 += (I8_5_A0[m] * d[m][c] + I8_5_A1[m] * a1[m][c]) * tp[m];
                    }
                    d[4][c] = n4 / (tp[3] * dt);
                    d[5][c] = n5 / (tp[3] * tp[2]);
                }
#pragma unroll
                for (int k = 0; k <= P; ++k) d[k][c] = a1[k][c];
                x[c] = x1[c];
                v[c] = v1[c];
                cx[c] = ncx[c];
                cv[c] = ncv[c];
            }
        }
        if (active) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                pos[c * n + li.g] = x[c];
                vel[c * n + li.g] = v[c];
                if constexpr (COMP) {
                    comp[c * n + li.g] = cx[c];
                    comp[n3 + c * n + li.g] = cv[c];
                }
#pragma unroll
                for (int k = 0; k < 2 * P; ++k) deriv[k * n3 + c * n + li.g] = d[k][c];
            }
        }
    }
}

template <int P, bool MIXED, bool COMP>
hipError_t run_pmc(const BatchPlan &pl, int corrector, int64_t n, const double *mass, double *pos, double *vel,
                   double *deriv, const double *dt_sys, int n_steps, int n_iter, const int *iters, double G,
                   double eps2, double *comp, int wg, hipStream_t st)
{
    const dim3 g(wg), b(kLanes);
    switch (corrector) {
        case 0: hipLaunchKernelGGL((batch_run_kernel<P, MIXED, 0, COMP>), g, b, 0, st, pl, n, mass, pos, vel, deriv, dt_sys, n_steps, n_iter, iters, G, eps2, comp); break;
        case 1: hipLaunchKernelGGL((batch_run_kernel<P, MIXED, 1, COMP>), g, b, 0, st, pl, n, mass, pos, vel, deriv, dt_sys, n_steps, n_iter, iters, G, eps2, comp); break;
        case 2: hipLaunchKernelGGL((batch_run_kernel<P, MIXED, 2, COMP>), g, b, 0, st, pl, n, mass, pos, vel, deriv, dt_sys, n_steps, n_iter, iters, G, eps2, comp); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Compensation is a template switch so that the plain kernel carries no
// compensation registers.
template <int P, bool MIXED>
hipError_t run_pm(const BatchPlan &pl, int corrector, int64_t n, const double *mass, double *pos, double *vel,
                  double *deriv, const double *dt_sys, int n_steps, int n_iter, const int *iters, double G,
                  double eps2, double *comp, int wg, hipStream_t st)
{
    return comp ? run_pmc<P, MIXED, true>(pl, corrector, n, mass, pos, vel, deriv, dt_sys, n_steps, n_iter, iters,
                                          G, eps2, comp, wg, st)
                : run_pmc<P, MIXED, false>(pl, corrector, n, mass, pos, vel, deriv, dt_sys, n_steps, n_iter, iters,
                                           G, eps2, comp, wg, st);
}

template <int K>
hipError_t init_pass(const BatchPlan &pl, int64_t n, const double *mass, const Path6 &path, int k_first, double G,
                     double eps2, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(batch_init_kernel<K>, dim3(pl.n_bins), dim3(kLanes), 0, st, pl, n, mass, path, k_first, G,
                       eps2, out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_reset_counter(int *counter, hipStream_t st)
{
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, st, counter);
    return hipGetLastError();
}

hipError_t launch_batch_init(const BatchPlan &pl, int p, int64_t n, const double *mass, const double *pos,
                             const double *vel, double *deriv, double G, double eps2, hipStream_t st)
{
    if (pl.n_bins <= 0 || n <= 0) return hipSuccess;
    const int64_t n3 = 3 * n;
    Path6 path{};
    path.p[0] = pos;
    path.p[1] = vel;
    for (int k = 0; k < 4; ++k) path.p[2 + k] = deriv + k * n3;
    hipError_t e = init_pass<1>(pl, n, mass, path, 0, G, eps2, deriv, st);
    if (e != hipSuccess || p < 2) return e;
    e = init_pass<3>(pl, n, mass, path, 2, G, eps2, deriv + 2 * n3, st);
    if (e != hipSuccess || p < 3) return e;
    return init_pass<5>(pl, n, mass, path, 4, G, eps2, deriv + 4 * n3, st);
}

hipError_t launch_batch_run(const BatchPlan &pl, int p, bool mixed, int corrector, int64_t n, const double *mass,
                            double *pos, double *vel, double *deriv, const double *dt_sys, int n_steps, int n_iter,
                            const int *iters, double G, double eps2, double *comp, int n_workgroups,
                            hipStream_t st)
{
    if (pl.n_bins <= 0 || n <= 0 || n_steps <= 0) return hipSuccess;
    if (n_workgroups < 1) n_workgroups = 1;
#define HERMITE_BATCH_CASE(PP)                                                                                     \
    case PP:                                                                                                       \
        return mixed ? run_pm<PP, true>(pl, corrector, n, mass, pos, vel, deriv, dt_sys, n_steps, n_iter, iters,   \
                                        G, eps2, comp, n_workgroups, st)                                                 \
                     : run_pm<PP, false>(pl, corrector, n, mass, pos, vel, deriv, dt_sys, n_steps, n_iter, iters,  \
                                         G, eps2, comp, n_workgroups, st);
    switch (p) {
        HERMITE_BATCH_CASE(1)
        HERMITE_BATCH_CASE(2)
        HERMITE_BATCH_CASE(3)
        default: return hipErrorInvalidValue;
    }
#undef HERMITE_BATCH_CASE
}

}  // namespace hermite
