// Batched form: thousands of independent small systems (1..64 bodies each)
// advanced for many P(EC)^n steps in ONE persistent kernel launch.
//
// Systems are packed first-fit-decreasing into 64-lane bins on the host (one
// lane slot per body).  Each workgroup holds W wave64 (W = 1, 2 or 4) that
// work on one bin at a time, taken from a device counter (bins are ordered
// longest first).  Every wave maps the bin's 64 slots onto its 64 lanes.
// The per-body work of a step (predictor, corrector, interpolation) is split
// by coordinate component: wave w keeps components w, w + W, ... of every
// body of the bin in VGPRs for all steps, so with W = 4 each lane holds one
// component of one body (wave 3 has none).  The O(N^2) evaluation is split by
// sweep step: every wave takes a contiguous share of the bin's sweep steps
// over the path of the current iterate, which sits in LDS.  The waves' sums
// meet in LDS and are added in wave order, so the result does not depend on
// timing.  The only global traffic per bin is the initial load, the final
// store and one counter increment.  An evaluation takes each pair of a system
// once, for both of its bodies (see the kernel); an idle lane, or a lane
// without a pair in a sweep step, contributes zero.  Systems may take
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


__global__ void reset_counter_kernel(int *counter) { counter[0] = 0; }

// Orders a wave's LDS accesses for the compiler: none is moved across it,
// whatever types they use (the segment sweep reads and writes the part array
// as float4 or double2 and elsewhere as double).  The hardware carries out one
// wave's LDS accesses in order, so this emits no instruction.
__device__ __forceinline__ void wave_lds_order()
{
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
}

__device__ constexpr double kInvB[9] = {0.0, 1.0, 1.0 / 2.0, 1.0 / 3.0, 1.0 / 4.0, 1.0 / 5.0, 1.0 / 6.0, 1.0 / 7.0, 1.0 / 8.0};

// The row CX[corrector][P][0..P+1] of the position corrector in use (a kernel
// argument, so one kernel serves every corrector).
struct CorrRow {
    double cx[kMaxP + 2];
};

template <int P, bool MIXED, bool COMP, int W>
__global__ __launch_bounds__(kLanes * W, 2) void batch_run_kernel(
    BatchPlan pl, int64_t n, const double *__restrict__ mass, double *__restrict__ pos, double *__restrict__ vel,
    double *__restrict__ deriv, const double *__restrict__ dt_sys, int n_steps, int n_iter,
    const int *__restrict__ iters, double G, double eps2, double *__restrict__ comp, CorrRow cr, int ring_min)
{
    constexpr int K = P;
    constexpr int NV = (K + 1) * 3;        // summed values per body: a^(0..K), 3 components each
    constexpr int NC = (3 + W - 1) / W;    // coordinate components per lane in the per-body work
    // chain arithmetic: FP64, or FP32 from the FP64 differences (mixed)
    using T = typename std::conditional<MIXED, float, double>::type;
    // the lone-wave kernel keeps two sweep steps in flight (one wave alone on
    // a SIMD is latency-bound); the 8th-order FP64 kernel with compensation
    // would exceed 256 registers with them
    constexpr bool kTwo = W == 1 && !(P == 3 && !MIXED && COMP);
    constexpr bool kEndInLoop = W >= 2;
    constexpr bool kLdsPass = W >= 2;   // j-side sums move through LDS (see the sweep)
    __shared__ double sp[NV][kLanes];      // path of the current iterate: [3 k + c][slot]
    __shared__ T sgm[kLanes];              // G m of every slot
    // each wave's sums over its sweep steps (a lone wave keeps them in
    // registers); during a segment sweep a wave's array carries the j-side
    // sums from lane to lane
    __shared__ __align__(16) double part[W == 1 ? 1 : W][W == 1 ? 1 : NV][W == 1 ? 1 : kLanes];
    __shared__ int next_bin;
    const int tid = threadIdx.x;
    // the wave index and every per-bin count below are the same in all lanes
    // of a wave; saying so keeps the sweep and iteration loops scalar
    const int w = __builtin_amdgcn_readfirstlane(tid / kLanes), l = tid % kLanes;
    const int64_t n3 = 3 * n;

    for (;;) {
        if (tid == 0) next_bin = atomicAdd(pl.counter, 1);
        __syncthreads();
        const int b = __builtin_amdgcn_readfirstlane(next_bin);
        __syncthreads();
        if (b >= pl.n_bins) break;
        const LaneInfo li = lane_info(pl, b, l, iters);
        const bool active = li.sys >= 0;
        const int maxlen = __builtin_amdgcn_readfirstlane(li.maxlen);
        // iterations of this bin and of this slot's system (the host checks
        // every count is in 1..64)
        const int bin_iter = iters ? __builtin_amdgcn_readfirstlane(li.maxiter) : n_iter;
        const int my_iter = (iters && active) ? iters[li.sys] : bin_iter;

        // the components this lane keeps: c = w + ci W, ci < NC, c < 3
        double x[NC], v[NC], d[2 * P][NC];
        // Kahan compensation of x and v (COMP, the option of Sec. 3.2): the
        // carried terms
        double cx[NC], cv[NC];
        double dt = 1.0;
        if (active) dt = dt_sys[li.sys];
#pragma unroll
        for (int ci = 0; ci < NC; ++ci) {
            const int c = w + ci * W;
            cx[ci] = cv[ci] = 0.0;
            if (c < 3 && active) {
                x[ci] = pos[c * n + li.g];
                v[ci] = vel[c * n + li.g];
                if constexpr (COMP) {
                    cx[ci] = comp[c * n + li.g];
                    cv[ci] = comp[n3 + c * n + li.g];
                }
#pragma unroll
                for (int k = 0; k < 2 * P; ++k) d[k][ci] = deriv[k * n3 + c * n + li.g];
            } else {
                x[ci] = 1.0e3 * (l + 1);   // far from every real body; contributes nothing (mass 0)
                v[ci] = 0.0;
#pragma unroll
                for (int k = 0; k < 2 * P; ++k) d[k][ci] = 0.0;
            }
        }
        if (w == 0) sgm[l] = (T)(active ? G * mass[li.g] : 0.0);
        // The bin's sweep (every pair of each system once, see below): its
        // kind, its step count, this wave's share of the steps [t0, t1], and
        // the lane a segment sweep passes sums from.
        const int sz = li.hi - li.lo, q = l - li.lo, half = sz / 2;
        const bool ring = maxlen >= ring_min;
        const int nsweep = ring ? min(maxlen - 1, kLanes / 2) : maxlen / 2;
        const int t0 = 1 + (w * nsweep) / W, t1 = ((w + 1) * nsweep) / W;
        const int succ = 4 * (li.lo + (q + 1 == sz ? 0 : q + 1));

        for (int step = 0; step < n_steps; ++step) {
            // dt is redefined here for the compiler: without it, the
            // predictor's, corrector's and interpolation's dt-derived factors
            // are hoisted out of the step loop and held in registers through
            // every sweep
            asm volatile("" : "+v"(dt));
            // Taylor predictor from the t0 state (Horner form) into the path.
#pragma unroll
            for (int ci = 0; ci < NC; ++ci) {
                const int c = w + ci * W;
                if (c >= 3) break;
                double xs[2 * P + 2];
                xs[0] = x[ci];
                xs[1] = v[ci];
#pragma unroll
                for (int k = 0; k < 2 * P; ++k) xs[k + 2] = d[k][ci];
#pragma unroll
                for (int f = 0; f <= K; ++f) {
                    const int M = 2 * P + 1 - f;
                    double s = xs[f + M];
#pragma unroll
                    for (int k = M - 1; k >= 0; --k) s = __builtin_fma(s, dt * kInvB[k + 1], xs[f + k]);
                    sp[3 * f + c][l] = s;
                }
            }
            // End of a system's step: interpolated higher derivatives
            // (R2), then the new state.  With several waves per bin it runs
            // inside the system's last iteration, so that nothing of the
            // correction stays live through later sweeps (fewer registers);
            // the lone-wave kernel, latency-bound on small systems, keeps the
            // last correction and ends every lane's step once after the
            // iterations (no divergent copies when systems of a bin take
            // different iteration counts).
            auto end_step = [&](int ci, const double (&a1)[K + 1], double x1, double v1, double ncx, double ncv) {
                if constexpr (P == 2) {
                    const double num = I6_A0[0] * d[0][ci] + I6_A1[0] * a1[0] +
                                       (I6_A0[1] * d[1][ci] + I6_A1[1] * a1[1]) * dt +
                                       (I6_A0[2] * d[2][ci] + I6_A1[2] * a1[2]) * (dt * dt);
                    d[3][ci] = num / (dt * dt * dt);
                }
                if constexpr (P == 3) {
                    const double tp[4] = {1.0, dt, dt * dt, dt * dt * dt};
                    double n4 = 0.0, n5 = 0.0;
#pragma unroll
                    for (int m = 0; m <= 3; ++m) {
                        n4 += (I8_4_A0[m] * d[m][ci] + I8_4_A1[m] * a1[m]) * tp[m];
                        n5 += (I8_5_A0[m] * d[m][ci] + I8_5_A1[m] * a1[m]) * tp[m];
                    }
                    d[4][ci] = n4 / (tp[3] * dt);
                    d[5][ci] = n5 / (tp[3] * tp[2]);
                }
#pragma unroll
                for (int k = 0; k <= P; ++k) d[k][ci] = a1[k];
                x[ci] = x1;
                v[ci] = v1;
                cx[ci] = ncx;
                cv[ci] = ncv;
            };
            struct Last {
                double a1[K + 1], x1, v1, ncx, ncv;
            };
            Last last[kEndInLoop ? 1 : NC];
            for (int it = 0; it < bin_iter; ++it) {
                // the start-of-step state is redefined here for the compiler,
                // so that no product of it is hoisted out of the iteration
                // loop and held in registers through the sweeps
#pragma unroll
                for (int ci = 0; ci < NC; ++ci) {
                    asm volatile("" : "+v"(x[ci]), "+v"(v[ci]));
#pragma unroll
                    for (int k = 0; k <= P; ++k) asm volatile("" : "+v"(d[k][ci]));
                }
                __syncthreads();   // the iterate's path is in sp; part is free
                // Evaluate a^(0..P) over each slot's own system, every pair
                // once; this wave takes sweep steps t0..t1.  A pair's chain
                // adds to the lane's own sums (the i-side) and, with the
                // opposite sign and the other mass, to the partner's (the
                // j-side).
                //  - ring: the whole wave is one ring; in step t lane l takes
                //    lane l + t (mod 64) if it is of the same system (at
                //    t = 32 only from lanes 0..31).  A system is contiguous,
                //    so each of its pairs is at ring distance
                //    <= min(maxlen - 1, 32) one way round.
                //  - segments: each system is a ring of its own; in step
                //    t = 1..sz/2 local body q takes q + t (mod sz) (at t = sz/2
                //    of an even sz only from its first half).
                double xi[K + 1][3];
#pragma unroll
                for (int k = 0; k <= K; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) xi[k][c] = sp[3 * k + c][l];
                const T gm_own = sgm[l];
                T acc[K + 1][3];
#pragma unroll
                for (int k = 0; k <= K; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) acc[k][c] = T(0);
                // one pair of this lane's body with slot jc: the i-side into
                // acc, the j-side into tj (no pair: zero differences, zero weight)
                auto pair = [&](int jc, bool act, T(&tj)[K + 1][3]) {
                    jc = act ? jc : l;
                    T r[3], vv[3], aa[3], jj[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        r[c] = (T)(sp[c][jc] - xi[0][c]);
                        vv[c] = (T)(sp[3 + c][jc] - xi[1][c]);
                        aa[c] = K >= 2 ? (T)(sp[K >= 2 ? 6 + c : c][jc] - xi[K >= 2 ? 2 : 0][c]) : T(0);
                        jj[c] = K >= 3 ? (T)(sp[K >= 3 ? 9 + c : c][jc] - xi[K >= 3 ? 3 : 0][c]) : T(0);
                    }
                    T w2 = fma_t(r[0], r[0], fma_t(r[1], r[1], fma_t(r[2], r[2], (T)eps2)));
                    w2 = act ? w2 : T(1);
                    const T rinv = rsqrt_t(w2);
                    const T rinv2 = rinv * rinv;
                    const T q3 = act ? rinv * rinv2 : T(0);
                    chain_pair<K, T>(r, vv, aa, jj, sgm[jc] * q3, -gm_own * q3, rinv2, acc, tj);
                };
                // The same pair in two parts, for the FP64 segment sweep: the
                // partner's path and G m are read first (into registers), the
                // chain runs later.  The mixed kernels keep the fused form
                // above, which stays within 168 registers (three waves per
                // SIMD).
                struct JPath {
                    double p[K + 1][3];
                    T gm;
                    bool act;
                };
                auto load_j = [&](int jc, bool act, JPath &jp) {
                    jc = act ? jc : l;
#pragma unroll
                    for (int k = 0; k <= K; ++k)
#pragma unroll
                        for (int c = 0; c < 3; ++c) jp.p[k][c] = sp[3 * k + c][jc];
                    jp.gm = sgm[jc];
                    jp.act = act;
                };
                auto pair_with = [&](const JPath &jp, T(&tj)[K + 1][3]) {
                    T r[3], vv[3], aa[3], jj[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        r[c] = (T)(jp.p[0][c] - xi[0][c]);
                        vv[c] = (T)(jp.p[1][c] - xi[1][c]);
                        aa[c] = K >= 2 ? (T)(jp.p[K >= 2 ? 2 : 0][c] - xi[K >= 2 ? 2 : 0][c]) : T(0);
                        jj[c] = K >= 3 ? (T)(jp.p[K >= 3 ? 3 : 0][c] - xi[K >= 3 ? 3 : 0][c]) : T(0);
                    }
                    T w2 = fma_t(r[0], r[0], fma_t(r[1], r[1], fma_t(r[2], r[2], (T)eps2)));
                    w2 = jp.act ? w2 : T(1);
                    const T rinv = rsqrt_t(w2);
                    const T rinv2 = rinv * rinv;
                    const T q3 = jp.act ? rinv * rinv2 : T(0);
                    chain_pair<K, T>(r, vv, aa, jj, jp.gm * q3, -gm_own * q3, rinv2, acc, tj);
                };
                T accj[K + 1][3];
#pragma unroll
                for (int k = 0; k <= K; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) accj[k][c] = T(0);
                // With several waves the j-side sums move between lanes
                // through the wave's own part array, which nothing else uses
                // between the barrier above and the totals written after the
                // sweep: every lane writes its sums at slot put and reads
                // those at slot get, two doubles or four floats per access
                // (a segment sweep's steps: put l, get the successor; the end
                // of every sweep: put the slot the sums belong to, get l).
                // The LDS carries out one wave's accesses in order, so the
                // reads see the writes without a workgroup barrier
                // (wave_lds_order only keeps the compiler from moving them).
                // The values are those of a lane-to-lane permute, but the LDS
                // unit takes these wide accesses faster than one permute per
                // 32-bit word.
                const int sl = succ >> 2;
                auto lds_pass = [&](int put, int get) {
                    if constexpr (!kLdsPass) return;   // a lone wave has no part array to pass through
                    T *f = &accj[0][0];
                    double *base = &part[W == 1 ? 0 : w][0][0];
                    if constexpr (MIXED) {
                        constexpr int NG = (NV + 3) / 4;   // fits: NG * 4 floats <= NV doubles
                        float4 *jb = reinterpret_cast<float4 *>(base);
#pragma unroll
                        for (int g = 0; g < NG; ++g) {
                            float4 v;
                            v.x = f[4 * g];
                            v.y = 4 * g + 1 < NV ? f[4 * g + 1] : 0.0f;
                            v.z = 4 * g + 2 < NV ? f[4 * g + 2] : 0.0f;
                            v.w = 4 * g + 3 < NV ? f[4 * g + 3] : 0.0f;
                            jb[g * kLanes + put] = v;
                        }
                        wave_lds_order();
#pragma unroll
                        for (int g = 0; g < NG; ++g) {
                            const float4 v = jb[g * kLanes + get];
                            f[4 * g] = v.x;
                            if (4 * g + 1 < NV) f[4 * g + 1] = v.y;
                            if (4 * g + 2 < NV) f[4 * g + 2] = v.z;
                            if (4 * g + 3 < NV) f[4 * g + 3] = v.w;
                        }
                    } else {
                        constexpr int NP = NV / 2;
                        double2 *jb = reinterpret_cast<double2 *>(base);
#pragma unroll
                        for (int g = 0; g < NP; ++g) jb[g * kLanes + put] = make_double2(f[2 * g], f[2 * g + 1]);
                        if constexpr ((NV & 1) != 0) base[(NV - 1) * kLanes + put] = f[NV - 1];
                        wave_lds_order();
#pragma unroll
                        for (int g = 0; g < NP; ++g) {
                            const double2 v = jb[g * kLanes + get];
                            f[2 * g] = v.x;
                            f[2 * g + 1] = v.y;
                        }
                        if constexpr ((NV & 1) != 0) f[NV - 1] = base[(NV - 1) * kLanes + get];
                    }
                    wave_lds_order();
                };
                // the sweep, RING a compile-time tag (one loop per kind)
                auto sweep = [&](auto ring_tag) {
                    constexpr bool RING = decltype(ring_tag)::value;
                    auto step_t = [&](int t) {
                        int jc;
                        bool act;
                        if constexpr (RING) {
                            jc = (l + t) & (kLanes - 1);
                            act = jc >= li.lo && jc < li.hi && !(t == kLanes / 2 && l >= kLanes / 2);
                        } else {
                            int q2 = q + t;
                            q2 = q2 >= sz ? q2 - sz : q2;
                            act = t <= half && !(2 * t == sz && q >= half);
                            jc = li.lo + q2;
                        }
                        pair(jc, act, accj);
                    };
                    auto pass_on = [&]() {
                        if constexpr (!RING && kLdsPass) {
                            lds_pass(l, sl);
                            return;
                        }
#pragma unroll
                        for (int k = 0; k <= K; ++k)
#pragma unroll
                            for (int c = 0; c < 3; ++c) {
                                if constexpr (RING) accj[k][c] = lane_down(accj[k][c]);
                                else accj[k][c] = lane_from(succ, accj[k][c]);
                            }
                    };
                    if (t0 <= t1) {
                        step_t(t0);
                        int t = t0 + 1;
                        if constexpr (kTwo) {
                            for (; t + 1 <= t1; t += 2) {
                                pass_on();
                                step_t(t);
                                pass_on();
                                step_t(t + 1);
                            }
                        }
                        for (; t <= t1; ++t) {
                            if constexpr (!RING && kLdsPass && !MIXED) {
                                // the partner's path is read before the pass,
                                // so that these reads do not queue behind it
                                // (FP64; the mixed kernel has no registers to
                                // spare for it at three waves per SIMD)
                                int q2 = q + t;
                                q2 = q2 >= sz ? q2 - sz : q2;
                                JPath jp;
                                load_j(li.lo + q2, t <= half && !(2 * t == sz && q >= half), jp);
                                pass_on();
                                pair_with(jp, accj);
                            } else {
                                pass_on();
                                step_t(t);
                            }
                        }
                    }
                };
                if (ring) sweep(std::true_type{});
                else sweep(std::false_type{});
                // lane l now holds the j-side sums of slot h: l + t1 (ring)
                // or local body q + t1 (segments); a wave without steps
                // holds zeros.  Every slot's j-side sums go to that slot's
                // lane and are added to its i-side sums:
                //  - several waves: through the wave's part array (each lane
                //    puts its sums at slot h and takes those of slot l), and
                //    the totals go to part for the component owners;
                //  - a lone wave: each lane takes them from the lane holding
                //    them, l - t1 (ring) or local body q - t1 (segments), by
                //    ds_bpermute, and keeps the totals in registers.
                double own[W == 1 ? K + 1 : 1][3];
                if constexpr (kLdsPass) {
                    lds_pass(ring ? ((l + t1) & (kLanes - 1)) : li.lo + (q + t1 % sz) % sz, l);
#pragma unroll
                    for (int k = 0; k <= K; ++k)
#pragma unroll
                        for (int c = 0; c < 3; ++c) part[w][3 * k + c][l] = (double)acc[k][c] + (double)accj[k][c];
                } else {
                    const int src = ring ? ((l - t1) & (kLanes - 1)) : li.lo + ((q - t1 % sz) % sz + sz) % sz;
#pragma unroll
                    for (int k = 0; k <= K; ++k)
#pragma unroll
                        for (int c = 0; c < 3; ++c) own[k][c] = (double)acc[k][c] + (double)lane_from(4 * src, accj[k][c]);
                }
                __syncthreads();   // every wave's sums are in part; sp may change
                // a system past its own iteration count keeps its last iterate
                if (it >= my_iter) continue;
                // Modified corrector for this lane's components: velocity
                // first, then position; the sums of the waves added in order.
                const bool fin = it + 1 == my_iter;
#pragma unroll
                for (int ci = 0; ci < NC; ++ci) {
                    const int c = w + ci * W;
                    if (c >= 3) break;
                    double a1[K + 1];
#pragma unroll
                    for (int k = 0; k <= K; ++k) {
                        if constexpr (W == 1) {
                            a1[k] = own[k][c];
                        } else {
                            double s = part[0][3 * k + c][l];
#pragma unroll
                            for (int u = 1; u < W; ++u) s += part[u][3 * k + c][l];
                            a1[k] = s;
                        }
                    }
                    double dv = 0.0;
#pragma unroll
                    for (int k = P; k >= 0; --k) {
                        const double s = (k & 1) ? (a1[k] - d[k][ci]) : (a1[k] + d[k][ci]);
                        dv = __builtin_fma(dv, dt, CV[P][k] * s);
                    }
                    double x1, v1, ncx = 0.0, ncv = 0.0;
                    if constexpr (COMP) {
                        const double y = dv * dt - cv[ci];
                        v1 = v[ci] + y;
                        ncv = (v1 - v[ci]) - y;
                    } else {
                        v1 = __builtin_fma(dv, dt, v[ci]);
                    }
                    double dx = 0.0;
#pragma unroll
                    for (int k = P + 1; k >= 1; --k) {
                        const double s = (k & 1) ? (a1[k - 1] - d[k - 1][ci]) : (a1[k - 1] + d[k - 1][ci]);
                        dx = __builtin_fma(dx, dt, cr.cx[k] * s);
                    }
                    dx = __builtin_fma(dx, dt, cr.cx[0] * (v1 + v[ci]));
                    if constexpr (COMP) {
                        const double y = dx * dt - cx[ci];
                        x1 = x[ci] + y;
                        ncx = (x1 - x[ci]) - y;
                    } else {
                        x1 = __builtin_fma(dx, dt, x[ci]);
                    }
                    if (!fin) {
                        sp[c][l] = x1;
                        sp[3 + c][l] = v1;
#pragma unroll
                        for (int m = 0; m <= K - 2; ++m) sp[3 * (2 + m) + c][l] = a1[m];
                    } else if constexpr (kEndInLoop) {
                        end_step(ci, a1, x1, v1, ncx, ncv);
                    } else {
#pragma unroll
                        for (int k = 0; k <= K; ++k) last[ci].a1[k] = a1[k];
                        last[ci].x1 = x1;
                        last[ci].v1 = v1;
                        last[ci].ncx = ncx;
                        last[ci].ncv = ncv;
                    }
                }
            }
            if constexpr (!kEndInLoop) {
#pragma unroll
                for (int ci = 0; ci < NC; ++ci) {
                    if (w + ci * W >= 3) break;
                    end_step(ci, last[ci].a1, last[ci].x1, last[ci].v1, last[ci].ncx, last[ci].ncv);
                }
            }
        }
        if (active) {
#pragma unroll
            for (int ci = 0; ci < NC; ++ci) {
                const int c = w + ci * W;
                if (c >= 3) break;
                pos[c * n + li.g] = x[ci];
                vel[c * n + li.g] = v[ci];
                if constexpr (COMP) {
                    comp[c * n + li.g] = cx[ci];
                    comp[n3 + c * n + li.g] = cv[ci];
                }
#pragma unroll
                for (int k = 0; k < 2 * P; ++k) deriv[k * n3 + c * n + li.g] = d[k][ci];
            }
        }
    }
}

template <int P, bool MIXED, bool COMP, int W>
hipError_t run_w(const BatchPlan &pl, const CorrRow &cr, int64_t n, const double *mass, double *pos, double *vel,
                 double *deriv, const double *dt_sys, int n_steps, int n_iter, const int *iters, double G,
                 double eps2, double *comp, const BatchShape &sh, hipStream_t st)
{
    hipLaunchKernelGGL((batch_run_kernel<P, MIXED, COMP, W>), dim3(sh.workgroups), dim3(kLanes * W), 0, st, pl, n,
                       mass, pos, vel, deriv, dt_sys, n_steps, n_iter, iters, G, eps2, comp, cr, sh.ring_min);
    return hipGetLastError();
}

// Compensation is a template switch so that the plain kernel carries no
// compensation registers.
template <int P, bool MIXED, bool COMP>
hipError_t run_pmc(const BatchPlan &pl, const CorrRow &cr, int64_t n, const double *mass, double *pos, double *vel,
                   double *deriv, const double *dt_sys, int n_steps, int n_iter, const int *iters, double G,
                   double eps2, double *comp, const BatchShape &sh, hipStream_t st)
{
    switch (sh.waves) {
        case 1: return run_w<P, MIXED, COMP, 1>(pl, cr, n, mass, pos, vel, deriv, dt_sys, n_steps, n_iter, iters, G, eps2, comp, sh, st);
        case 2: return run_w<P, MIXED, COMP, 2>(pl, cr, n, mass, pos, vel, deriv, dt_sys, n_steps, n_iter, iters, G, eps2, comp, sh, st);
        case 4: return run_w<P, MIXED, COMP, 4>(pl, cr, n, mass, pos, vel, deriv, dt_sys, n_steps, n_iter, iters, G, eps2, comp, sh, st);
        default: return hipErrorInvalidValue;
    }
}

template <int P, bool MIXED>
hipError_t run_pm(const BatchPlan &pl, const CorrRow &cr, int64_t n, const double *mass, double *pos, double *vel,
                  double *deriv, const double *dt_sys, int n_steps, int n_iter, const int *iters, double G,
                  double eps2, double *comp, const BatchShape &sh, hipStream_t st)
{
    return comp ? run_pmc<P, MIXED, true>(pl, cr, n, mass, pos, vel, deriv, dt_sys, n_steps, n_iter, iters, G, eps2,
                                          comp, sh, st)
                : run_pmc<P, MIXED, false>(pl, cr, n, mass, pos, vel, deriv, dt_sys, n_steps, n_iter, iters, G, eps2,
                                           comp, sh, st);
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

namespace {
template <int P, bool MIXED, bool COMP, int W>
int resident_w()
{
    int per_cu = 0;
    const hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_run_kernel<P, MIXED, COMP, W>, kLanes * W, 0);
    return e == hipSuccess ? per_cu : 0;
}

template <int P, bool MIXED, bool COMP>
int resident_pmc(const BatchShape &sh)
{
    switch (sh.waves) {
        case 1: return resident_w<P, MIXED, COMP, 1>();
        case 2: return resident_w<P, MIXED, COMP, 2>();
        case 4: return resident_w<P, MIXED, COMP, 4>();
        default: return 0;
    }
}

template <int P>
int resident_p(const BatchShape &sh, bool mixed, bool comp)
{
    if (mixed) return comp ? resident_pmc<P, true, true>(sh) : resident_pmc<P, true, false>(sh);
    return comp ? resident_pmc<P, false, true>(sh) : resident_pmc<P, false, false>(sh);
}
}  // namespace

int batch_resident_per_cu(const BatchShape &sh, int p, bool mixed, bool comp)
{
    switch (p) {
        case 1: return resident_p<1>(sh, mixed, comp);
        case 2: return resident_p<2>(sh, mixed, comp);
        case 3: return resident_p<3>(sh, mixed, comp);
        default: return 0;
    }
}

bool batch_shape_ok(const BatchShape &sh)
{
    return sh.workgroups >= 1 && (sh.waves == 1 || sh.waves == 2 || sh.waves == 4) && sh.ring_min >= 2;
}

hipError_t launch_batch_run(const BatchPlan &pl, int p, bool mixed, int corrector, int64_t n, const double *mass,
                            double *pos, double *vel, double *deriv, const double *dt_sys, int n_steps, int n_iter,
                            const int *iters, double G, double eps2, double *comp, const BatchShape &shape,
                            hipStream_t st)
{
    if (pl.n_bins <= 0 || n <= 0 || n_steps <= 0) return hipSuccess;
    if (!batch_shape_ok(shape) || corrector < 0 || corrector > 2 || p < 1 || p > 3) return hipErrorInvalidValue;
    CorrRow cr{};
    for (int k = 0; k <= p + 1; ++k) cr.cx[k] = CX[corrector][p][k];
#define HERMITE_BATCH_CASE(PP)                                                                                     \
    case PP:                                                                                                       \
        return mixed ? run_pm<PP, true>(pl, cr, n, mass, pos, vel, deriv, dt_sys, n_steps, n_iter, iters, G, eps2, \
                                        comp, shape, st)                                                           \
                     : run_pm<PP, false>(pl, cr, n, mass, pos, vel, deriv, dt_sys, n_steps, n_iter, iters, G,      \
                                         eps2, comp, shape, st);
    switch (p) {
        HERMITE_BATCH_CASE(1)
        HERMITE_BATCH_CASE(2)
        HERMITE_BATCH_CASE(3)
        default: return hipErrorInvalidValue;
    }
#undef HERMITE_BATCH_CASE
}

}  // namespace hermite
