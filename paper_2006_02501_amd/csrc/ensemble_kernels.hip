// Ensemble form: independent systems of 2..128 bodies, each integrated by
// ONE workgroup with the variable, time-symmetric step of Sec. 3.3 (Eq. 25)
// from its current time to its end time, without returning to the host
// (the paper's N-body test, Table 1, is a 101-body system run for ~10^5 to
// 10^6 such steps; one launch carries a whole grid of them, one system per
// CU).
//
// A workgroup is 512 threads (8 wave64).  Thread t takes the i-slot
// t % NI and the j-part t / NI, NI = 64 or 128 (the system's size rounded up
// to whole waves), so 8 or 4 threads share an i-particle and split its
// j-range.  Every thread of an i-slot keeps the same copy of that particle's
// state (x, v, a^(0..2p-1)) in VGPRs and runs the per-particle predictor and
// corrector itself (O(N) work, repeated, so no broadcast is needed); the
// evaluation's j-part sums and the pair-rate maxima meet in LDS and are
// added in a fixed order, so every thread forms the same a and the same
// step, and the results do not depend on timing.
//
// Per step: prediction with dt = H_-, a pair-rate pass at the predicted
// positions for H_+ there and the prediction redone for dt = (H_- + H_+)/2;
// then n times (evaluation at t0 + dt with the pair rate fused in, correction
// with that dt, and before the last iteration the next dt = (H_- + H_+)/2
// from H_+ at this evaluation point, the iterate being moved to the new end
// point along its Taylor series); the interpolated a^(p+1..2p-1); then one
// pass at the new x for the next H_- and, once t is past the recording time,
// the energy.
#include "hermite_coeffs.h"
#include "kernels.h"
#include "pair_chain.h"

namespace hermite {
namespace {

constexpr int kEnsThreads = 512;
constexpr int kEnsWaves = kEnsThreads / 64;
constexpr int kEnsMaxN = 128;

__device__ constexpr double kInvE[9] = {0.0, 1.0, 1.0 / 2.0, 1.0 / 3.0, 1.0 / 4.0, 1.0 / 5.0, 1.0 / 6.0, 1.0 / 7.0, 1.0 / 8.0};

struct Slots {
    int N;       // bodies of this system
    int NI;      // i-slots (64 or 128)
    int JP;      // j-parts (8 or 4)
    int islot, jp;
    bool live;   // islot < N
    int jb, je;  // this thread's j-range
    int64_t g;   // global index of this thread's i-particle
};

__device__ __forceinline__ Slots slots_of(const int64_t *offsets, int sys, int tid)
{
    Slots s;
    const int64_t off = offsets[sys];
    s.N = (int)(offsets[sys + 1] - off);
    s.NI = s.N <= 64 ? 64 : 128;
    s.JP = kEnsThreads / s.NI;
    s.islot = tid % s.NI;
    s.jp = tid / s.NI;
    s.live = s.islot < s.N;
    const int chunk = (s.N + s.JP - 1) / s.JP;
    s.jb = min(s.N, s.jp * chunk);
    s.je = min(s.N, s.jb + chunk);
    s.g = off + (s.live ? s.islot : 0);
    return s;
}

// Wave-wide max (a NaN is dropped) and sum by xor-shuffle trees (a fixed
// order); the 8 wave results then meet in LDS, also in a fixed order.
__device__ __forceinline__ double wave_max(double q)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) q = __builtin_fmax(q, __shfl_xor(q, off, 64));
    return q;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Generic-order initialisation pass K (1, 3, 5) for every system: outputs
// k_first..K of the pair derivatives along path (x^(0..K) of all bodies).
template <int K>
__global__ __launch_bounds__(kEnsThreads) void ens_init_kernel(const int64_t *__restrict__ offsets, int64_t n,
                                                               const double *__restrict__ mass, Path6Ptr path,
                                                               int k_first, double G, double eps2,
                                                               double *__restrict__ out)
{
    __shared__ double sp[K + 1][3][kEnsMaxN];
    __shared__ double sm[kEnsMaxN];
    __shared__ double red[8][3][64];
    const int tid = threadIdx.x;
    const Slots s = slots_of(offsets, blockIdx.x, tid);
    if (s.jp == 0) {
        sm[s.islot] = s.live ? G * mass[s.g] : 0.0;
#pragma unroll
        for (int k = 0; k <= K; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) sp[k][c][s.islot] = s.live ? path.p[k][c * n + s.g] : 0.0;
    }
    __syncthreads();
    double xi[K + 1][3], acc[K + 1][3];
#pragma unroll
    for (int k = 0; k <= K; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xi[k][c] = sp[k][c][s.islot];
            acc[k][c] = 0.0;
        }
    for (int j = s.jb; j < s.je; ++j) {
        const bool skip = !s.live || j == s.islot;
        double r[K + 1][3];
#pragma unroll
        for (int k = 0; k <= K; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) r[k][c] = sp[k][c][j] - xi[k][c];
        generic_accumulate<K>(r, eps2, sm[j], skip, acc);
    }
    // j-part sums meet in LDS, one order and one 64-slot group at a time,
    // added in j-part order (runs once per run, so the barriers do not matter)
#pragma unroll
    for (int k = 0; k <= K; ++k) {
        if (k < k_first) continue;
        for (int grp = 0; grp < s.NI / 64; ++grp) {
            __syncthreads();
            if (s.islot / 64 == grp) {
#pragma unroll
                for (int c = 0; c < 3; ++c) red[s.jp][c][s.islot % 64] = acc[k][c];
            }
            __syncthreads();
            if (s.jp == 0 && s.islot / 64 == grp && s.live) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    double t = red[0][c][s.islot % 64];
                    for (int q = 1; q < s.JP; ++q) t += red[q][c][s.islot % 64];
                    out[((int64_t)(k - k_first) * 3 + c) * n + s.g] = t;
                }
            }
        }
    }
}

// Pair pass at positions sp[0] (all bodies of the system in LDS): this
// thread's maximum pair rate and, when want_pot, its part of sum_j G m_j / r.
__device__ __forceinline__ void rate_pass(const Slots &s, const double (*sp0)[kEnsMaxN], const double *sm,
                                          const double (&xi)[3], double gmi, double eps2, bool want_pot,
                                          double &q, double &pot)
{
    q = 0.0;
    pot = 0.0;
#pragma unroll 4
    for (int j = s.jb; j < s.je; ++j) {
        const double dx = sp0[0][j] - xi[0], dy = sp0[1][j] - xi[1], dz = sp0[2][j] - xi[2];
        const double w = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
        const bool self = j == s.islot || !s.live;
        const double y = rsqrt64(self ? 1.0 : w);
        const double gm = self ? 0.0 : sm[j];
        q = __builtin_fmax(q, (gmi + gm) * (self ? 0.0 : y * y * y));
        if (want_pot) pot = __builtin_fma(gm, y, pot);
    }
}

template <int P, int CORR>
__global__ __launch_bounds__(kEnsThreads) void ens_run_kernel(EnsembleArgs a)
{
    constexpr int K = P;
    __shared__ double sp[K + 1][3][kEnsMaxN];
    __shared__ double sm[kEnsMaxN];
    // j-part sums, [order*3 + component][j-part][i-slot]
    __shared__ double red[(K + 1) * 3 * kEnsThreads];
    __shared__ double rq[kEnsWaves], re[kEnsWaves];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int sys = blockIdx.x;
    const Slots s = slots_of(a.offsets, sys, tid);
    const int64_t n = a.n, n3 = 3 * n;
    const EnsembleCfg cfg = a.cfg[sys];
    EnsembleStatus st = a.status[sys];
    if (st.failed) return;

    double x[3], v[3], d[2 * P][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        x[c] = s.live ? a.pos[c * n + s.g] : 0.0;
        v[c] = s.live ? a.vel[c * n + s.g] : 0.0;
#pragma unroll
        for (int k = 0; k < 2 * P; ++k) d[k][c] = s.live ? a.deriv[k * n3 + c * n + s.g] : 0.0;
    }
    const double mi = s.live ? a.mass[s.g] : 0.0;
    const double gmi = a.G * mi;
    if (s.jp == 0) sm[s.islot] = gmi;

    // Barriers.  LDS is written in three places -- the iterate's path (sp),
    // the j-part sums and wave maxima (red, rq), and the positions for a
    // criterion pass (sp[0]) -- each right after a barrier that every read of
    // the previous contents precedes, and read after the one barrier that
    // follows the writes.  So an iteration takes two barriers and each
    // criterion pass (at the predicted end point, and at the new x after the
    // step) two.
    //
    // positions into LDS, then a criterion pass at them (with the energy, for
    // E0 on a system's first call and for the records)
    auto share_pos = [&](const double (&xs)[3]) {
        if (s.jp == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) sp[0][c][s.islot] = xs[c];
        }
        __syncthreads();
    };
    auto energy_and_rate = [&](const double (&xs)[3], bool want_pot, double &qmax, double &E) {
        double q, pot;
        rate_pass(s, sp[0], sm, xs, gmi, a.eps2, want_pot, q, pot);
        const double qw = wave_max(q);
        double ew = 0.0;
        if (want_pot) {
            const double kin = (s.jp == 0 && s.live) ? 0.5 * mi * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) : 0.0;
            ew = wave_sum(kin - 0.5 * mi * pot);
        }
        if (lane == 0) {
            rq[wave] = qw;
            re[wave] = ew;
        }
        __syncthreads();
        qmax = rq[0];
        E = re[0];
#pragma unroll
        for (int w = 1; w < kEnsWaves; ++w) {
            qmax = __builtin_fmax(qmax, rq[w]);
            E += re[w];
        }
    };

    share_pos(x);   // (its barrier also publishes sm)
    double qm, E;
    const bool first = st.steps == 0;
    energy_and_rate(x, first, qm, E);
    if (first) st.E0 = E;
    double Hm = cfg.eta / sqrt(qm);
    double t = st.t;
    int64_t steps_here = 0;
    bool failed = !(Hm > 0.0) || !__builtin_isfinite(Hm);

    while (!failed && t < cfg.t_end && steps_here < a.max_steps) {
        double dt = Hm;
        // predictor (Horner form, every stored derivative) for a step dt
        double path[K + 1][3];
        auto predict_to = [&](double dt_p) {
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
                    double acc_ = xs[f + M];
#pragma unroll
                    for (int k = M - 1; k >= 0; --k) acc_ = __builtin_fma(acc_, dt_p * kInvE[k + 1], xs[f + k]);
                    path[f][c] = acc_;
                }
            }
        };
        // H_+ at the end point predicted for dt = H_-, then dt = (H_- + H_+)/2
        predict_to(Hm);
        {
            double qp, unused;
            const double xp[3] = {path[0][0], path[0][1], path[0][2]};
            share_pos(xp);
            energy_and_rate(xp, false, qp, unused);
            const double Hp = cfg.eta / sqrt(qp);
            if (!(Hp > 0.0) || !__builtin_isfinite(Hp)) {
                failed = true;
                break;
            }
            dt = 0.5 * (Hm + Hp);
        }
        predict_to(dt);
        double a1[K + 1][3], x1[3], v1[3];
        for (int it = 0; it < cfg.n_iter; ++it) {
            if (s.jp == 0) {
#pragma unroll
                for (int k = 0; k <= K; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) sp[k][c][s.islot] = path[k][c];
            }
            __syncthreads();
            double acc[K + 1][3];
#pragma unroll
            for (int k = 0; k <= K; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[k][c] = 0.0;
            double q = 0.0;
            // two pairs in flight where the registers allow it (not at 8th order)
            constexpr int kUnr = K >= 3 ? 1 : 2;
#pragma unroll kUnr
            for (int j = s.jb; j < s.je; ++j) {
                double r[3], vv[3], aa[3], jj[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    r[c] = sp[0][c][j] - path[0][c];
                    vv[c] = sp[1][c][j] - path[1][c];
                    aa[c] = K >= 2 ? sp[K >= 2 ? 2 : 0][c][j] - path[K >= 2 ? 2 : 0][c] : 0.0;
                    jj[c] = K >= 3 ? sp[K >= 3 ? 3 : 0][c][j] - path[K >= 3 ? 3 : 0][c] : 0.0;
                }
                const bool self = j == s.islot || !s.live;
                double w = __builtin_fma(r[0], r[0], __builtin_fma(r[1], r[1], __builtin_fma(r[2], r[2], a.eps2)));
                w = self ? 1.0 : w;
                const double m = self ? 0.0 : sm[j];
                const double rinv = rsqrt64(w);
                const double rinv2 = rinv * rinv;
                const double r3 = self ? 0.0 : rinv * rinv2;
                chain_accumulate<K, double>(r, vv, aa, jj, m * r3, rinv2, acc);
                q = __builtin_fmax(q, (gmi + m) * r3);
            }
            // j-part sums added in j-part order; the block's largest pair rate
#pragma unroll
            for (int k = 0; k <= K; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) red[((k * 3 + c) * s.JP + s.jp) * s.NI + s.islot] = acc[k][c];
            const double qw = wave_max(q);
            if (lane == 0) rq[wave] = qw;
            __syncthreads();
#pragma unroll
            for (int k = 0; k <= K; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double *rr = red + (k * 3 + c) * s.JP * s.NI + s.islot;
                    double tsum = rr[0];
                    for (int p2 = 1; p2 < s.JP; ++p2) tsum += rr[p2 * s.NI];
                    a1[k][c] = tsum;
                }
            // modified corrector with this iteration's dt: velocity first, then position
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double dv = 0.0;
#pragma unroll
                for (int k = P; k >= 0; --k) {
                    const double sg = (k & 1) ? (a1[k][c] - d[k][c]) : (a1[k][c] + d[k][c]);
                    dv = __builtin_fma(dv, dt, CV[P][k] * sg);
                }
                v1[c] = __builtin_fma(dv, dt, v[c]);
                double dx = 0.0;
#pragma unroll
                for (int k = P + 1; k >= 1; --k) {
                    const double sg = (k & 1) ? (a1[k - 1][c] - d[k - 1][c]) : (a1[k - 1][c] + d[k - 1][c]);
                    dx = __builtin_fma(dx, dt, CX[CORR][P][k] * sg);
                }
                dx = __builtin_fma(dx, dt, CX[CORR][P][0] * (v1[c] + v[c]));
                x1[c] = __builtin_fma(dx, dt, x[c]);
            }
            if (it + 1 < cfg.n_iter) {
                // the next dt from H_+ at this evaluation point; the iterate,
                // moved to t0 + next dt along its Taylor series
                // (x1, v1, a1^(0..P)), is the next path
                double qb = rq[0];
#pragma unroll
                for (int w = 1; w < kEnsWaves; ++w) qb = __builtin_fmax(qb, rq[w]);
                const double Hp = cfg.eta / sqrt(qb);
                if (!(Hp > 0.0) || !__builtin_isfinite(Hp)) {
                    failed = true;
                    break;
                }
                const double dtn = 0.5 * (Hm + Hp);
                const double sh = dtn - dt;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    double xs[P + 3];
                    xs[0] = x1[c];
                    xs[1] = v1[c];
#pragma unroll
                    for (int k = 0; k <= P; ++k) xs[k + 2] = a1[k][c];
#pragma unroll
                    for (int f = 0; f <= K; ++f) {
                        double acc_ = xs[P + 2];
#pragma unroll
                        for (int k = P + 1 - f; k >= 0; --k) acc_ = __builtin_fma(acc_, sh * kInvE[k + 1], xs[f + k]);
                        path[f][c] = acc_;
                    }
                }
                dt = dtn;
            }
        }
        if (failed) break;
        // end of step: interpolated higher derivatives, the new state
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
                for (int m2 = 0; m2 <= 3; ++m2) {
                    n4 += (I8_4_A0[m2] * d[m2][c] + I8_4_A1[m2] * a1[m2][c]) * tp[m2];
                    n5 += (I8_5_A0[m2] * d[m2][c] + I8_5_A1[m2] * a1[m2][c]) * tp[m2];
                }
                d[4][c] = n4 / (tp[3] * dt);
                d[5][c] = n5 / (tp[3] * tp[2]);
            }
#pragma unroll
            for (int k = 0; k <= P; ++k) d[k][c] = a1[k][c];
            x[c] = x1[c];
            v[c] = v1[c];
        }
        t += dt;
        ++steps_here;
        // next H_- at the new positions, with the energy once past rec_from
        const bool rec = t > cfg.rec_from;
        share_pos(x);
        energy_and_rate(x, rec, qm, E);
        Hm = cfg.eta / sqrt(qm);
        failed = !(Hm > 0.0) || !__builtin_isfinite(Hm);
        if (rec) {
            if (st.records < a.rec_cap && tid == 0) {
                double *r = a.rec + ((int64_t)sys * a.rec_cap + st.records) * 2;
                r[0] = t;
                r[1] = E;
            }
            if (st.records < a.rec_cap) ++st.records;
            else st.rec_overflow = 1;
        }
    }
    if (s.live && s.jp == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            a.pos[c * n + s.g] = x[c];
            a.vel[c * n + s.g] = v[c];
#pragma unroll
            for (int k = 0; k < 2 * P; ++k) a.deriv[k * n3 + c * n + s.g] = d[k][c];
        }
    }
    if (tid == 0) {
        st.t = t;
        st.steps += steps_here;
        st.failed = failed ? 1 : 0;
        a.status[sys] = st;
    }
}

}  // namespace

hipError_t launch_ensemble_init(const int64_t *offsets, int32_t n_sys, int p, int64_t n, const double *mass,
                                const double *pos, const double *vel, double *deriv, double G, double eps2,
                                hipStream_t st)
{
    if (n_sys <= 0 || n <= 0) return hipSuccess;
    const int64_t n3 = 3 * n;
    Path6Ptr path{};
    path.p[0] = pos;
    path.p[1] = vel;
    for (int k = 0; k < 4; ++k) path.p[2 + k] = deriv + k * n3;
    hipLaunchKernelGGL(ens_init_kernel<1>, dim3(n_sys), dim3(kEnsThreads), 0, st, offsets, n, mass, path, 0, G,
                       eps2, deriv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || p < 2) return e;
    hipLaunchKernelGGL(ens_init_kernel<3>, dim3(n_sys), dim3(kEnsThreads), 0, st, offsets, n, mass, path, 2, G,
                       eps2, deriv + 2 * n3);
    e = hipGetLastError();
    if (e != hipSuccess || p < 3) return e;
    hipLaunchKernelGGL(ens_init_kernel<5>, dim3(n_sys), dim3(kEnsThreads), 0, st, offsets, n, mass, path, 4, G,
                       eps2, deriv + 4 * n3);
    return hipGetLastError();
}

hipError_t launch_ensemble_run(const EnsembleArgs &a, int p, int corrector, hipStream_t st)
{
    if (a.n_sys <= 0) return hipSuccess;
    const dim3 g(a.n_sys), b(kEnsThreads);
#define HERMITE_ENS_CASE(PP, CC) \
    if (p == PP && corrector == CC) { hipLaunchKernelGGL((ens_run_kernel<PP, CC>), g, b, 0, st, a); return hipGetLastError(); }
    HERMITE_ENS_CASE(1, 0) HERMITE_ENS_CASE(1, 1) HERMITE_ENS_CASE(1, 2)
    HERMITE_ENS_CASE(2, 0) HERMITE_ENS_CASE(2, 1) HERMITE_ENS_CASE(2, 2)
    HERMITE_ENS_CASE(3, 0) HERMITE_ENS_CASE(3, 1) HERMITE_ENS_CASE(3, 2)
#undef HERMITE_ENS_CASE
    return hipErrorInvalidValue;
}

}  // namespace hermite
