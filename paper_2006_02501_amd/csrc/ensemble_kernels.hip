// Ensemble form: independent systems of 2..128 bodies, each integrated by
// ONE workgroup with the variable, time-symmetric step of Sec. 3.3 (Eq. 25)
// from its current time to its end time, without returning to the host
// (the paper's N-body test, Table 1, is a 101-body system run for ~10^5 to
// 10^6 such steps; one launch carries a whole grid of them, one system per
// CU).
//
// A workgroup is 1024 threads (16 wave64, four per SIMD).  The state of the
// system (x, v, a^(0..2p-1) of every body) lives in LDS; the per-body work
// (predictor, corrector, the shift of the iterate, the interpolation) runs
// once per (body, component) on the owner threads tid < 3N.  For the
// evaluation thread t takes the i-slot t % N and the j-part t / N of the
// j-range; the j-part sums and the pair-rate maxima meet in LDS and are added
// in a fixed order, so every thread forms the same step and the results do
// not depend on timing.  (The initialisation passes, run once, use 512
// threads and 64 or 128 slots.)
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

constexpr int kEnsInitThreads = 512;    // the initialisation passes (once per run)
constexpr int kEnsThreads = 1024;       // the run kernel: 16 wave64, four per SIMD
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

// exact: as many i-slots as bodies (threads beyond JP NI take no pairs);
// else 64 or 128 slots, the system's size rounded up to whole waves.
__device__ __forceinline__ Slots slots_of(const int64_t *offsets, int sys, int tid, int threads, bool exact)
{
    Slots s;
    const int64_t off = offsets[sys];
    s.N = (int)(offsets[sys + 1] - off);
    s.NI = exact ? s.N : s.N <= 64 ? 64 : 128;
    s.JP = threads / s.NI;
    s.islot = tid % s.NI;
    s.jp = tid / s.NI;
    s.live = s.islot < s.N && s.jp < s.JP;
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
__global__ __launch_bounds__(kEnsInitThreads) void ens_init_kernel(const int64_t *__restrict__ offsets, int64_t n,
                                                               const double *__restrict__ mass, Path6Ptr path,
                                                               int k_first, double G, double eps2,
                                                               double *__restrict__ out)
{
    __shared__ double sp[K + 1][3][kEnsMaxN];
    __shared__ double sm[kEnsMaxN];
    __shared__ double red[8][3][64];
    const int tid = threadIdx.x;
    const Slots s = slots_of(offsets, blockIdx.x, tid, kEnsInitThreads, false);
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

// Pair pass at positions (X, Y, Z)[slot] (all bodies of the system in LDS):
// this thread's maximum pair rate and, when want_pot, its part of
// sum_j G m_j / r.
__device__ __forceinline__ void rate_pass(const Slots &s, const double *X, const double *Y, const double *Z,
                                          const double *sm, double gmi, double eps2, bool want_pot, double &q,
                                          double &pot)
{
    const double xi0 = X[s.islot], xi1 = Y[s.islot], xi2 = Z[s.islot];
    q = 0.0;
    pot = 0.0;
#pragma unroll 4
    for (int j = s.jb; j < s.je; ++j) {
        const double dx = X[j] - xi0, dy = Y[j] - xi1, dz = Z[j] - xi2;
        const double w = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
        const bool self = j == s.islot || !s.live;
        const double y = rsqrt64(self ? 1.0 : w);
        const double gm = self ? 0.0 : sm[j];
        q = __builtin_fmax(q, (gmi + gm) * (self ? 0.0 : y * y * y));
        if (want_pot) pot = __builtin_fma(gm, y, pot);
    }
}

// One system per workgroup of 1024 threads.  The per-body state x, v,
// a^(0..2P-1) lives in LDS, and the per-body work (predictor, corrector,
// shift of the iterate, interpolation) is done once per (body, component) by
// the "owner" threads tid < 3 NI (slot tid % NI, component tid / NI).  The
// evaluation is spread over all threads: thread t takes i-slot t % NI and the
// j-part t / NI of the j-range (16 or 8 j-parts), with the i-path read from
// LDS; its sums go to LDS and each owner adds the j-parts of its component in
// j-part order.  Keeping the state out of the registers is what lets four
// waves share a SIMD.
template <int P, int CORR>
__global__ __launch_bounds__(kEnsThreads) void ens_run_kernel(EnsembleArgs a)
{
    constexpr int K = P;
    constexpr int NS = 2 + 2 * P;          // state per component: x, v, a^(0..2P-1)
    __shared__ double sp[K + 1][3][kEnsMaxN];       // path of the current iterate
    __shared__ double stl[3][NS][kEnsMaxN];          // state, [component][x, v, a^(k)][slot]
    __shared__ double sm[kEnsMaxN];
    // j-part sums, [order*3 + component][j-part * NI + i-slot]
    __shared__ double red[(K + 1) * 3][kEnsThreads];
    __shared__ double rq[kEnsWaves], re[kEnsWaves];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int sys = blockIdx.x;
    const Slots s = slots_of(a.offsets, sys, tid, kEnsThreads, true);
    const int64_t n = a.n, n3 = 3 * n;
    const int64_t off = a.offsets[sys];
    const EnsembleCfg cfg = a.cfg[sys];
    EnsembleStatus st = a.status[sys];
    if (st.failed) return;

    // owner threads: (slot, component)
    const bool owner = tid < 3 * s.NI;
    const int oslot = tid % s.NI, oc = owner ? tid / s.NI : 0;
    const bool olive = owner && oslot < s.N;
    if (owner) {
#pragma unroll
        for (int f = 0; f < NS; ++f) {
            double val = 0.0;
            if (olive) {
                const int64_t g = off + oslot;
                val = f == 0 ? a.pos[oc * n + g] : f == 1 ? a.vel[oc * n + g] : a.deriv[(f - 2) * n3 + oc * n + g];
            }
            stl[oc][f][oslot] = val;
        }
    }
    const double mi = s.live ? a.mass[s.g] : 0.0;
    const double gmi = a.G * mi;
    if (s.jp == 0) sm[s.islot] = gmi;

    // Barriers.  LDS is written in four places -- the state (stl, by the
    // owners at the end of a step), the path (sp), the j-part sums and wave
    // maxima (red, rq, re) -- each right after a barrier that every read of
    // the previous contents precedes, and read after the barrier that
    // follows the writes.
    //
    // A criterion pass at the positions xs: the largest pair rate and, when
    // want_pot, the energy (kinetic part from the state's v)
    auto energy_and_rate = [&](const double *X, const double *Y, const double *Z, bool want_pot, double &qmax,
                               double &E) {
        double q, pot;
        rate_pass(s, X, Y, Z, sm, gmi, a.eps2, want_pot, q, pot);
        const double qw = wave_max(q);
        double ew = 0.0;
        if (want_pot) {
            double kin = 0.0;
            if (s.jp == 0 && s.live) {
                const double v0 = stl[0][1][s.islot], v1 = stl[1][1][s.islot], v2 = stl[2][1][s.islot];
                kin = 0.5 * mi * (v0 * v0 + v1 * v1 + v2 * v2);
            }
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
    // the owner's predictor: path f of component oc for a step dt_p
    auto predict_f = [&](double dt_p, int f) {
        const int M = 2 * P + 1 - f;
        double acc_ = stl[oc][f + M][oslot];
#pragma unroll
        for (int k = M - 1; k >= 0; --k) acc_ = __builtin_fma(acc_, dt_p * kInvE[k + 1], stl[oc][f + k][oslot]);
        return acc_;
    };

    __syncthreads();   // the state and sm are in LDS
    double qm, E;
    const bool first = st.steps == 0;
    energy_and_rate(stl[0][0], stl[1][0], stl[2][0], first, qm, E);
    if (first) st.E0 = E;
    double Hm = cfg.eta / sqrt(qm);
    double t = st.t;
    int64_t steps_here = 0;
    bool failed = !(Hm > 0.0) || !__builtin_isfinite(Hm);

    while (!failed && t < cfg.t_end && steps_here < a.max_steps) {
        // H_+ at the end point predicted for dt = H_-, then dt = (H_- + H_+)/2
        if (owner) sp[0][oc][oslot] = predict_f(Hm, 0);
        __syncthreads();
        double dt;
        {
            double qp, unused;
            energy_and_rate(sp[0][0], sp[0][1], sp[0][2], false, qp, unused);
            const double Hp = cfg.eta / sqrt(qp);
            if (!(Hp > 0.0) || !__builtin_isfinite(Hp)) {
                failed = true;
                break;
            }
            dt = 0.5 * (Hm + Hp);
        }
        if (owner) {
#pragma unroll
            for (int f = 0; f <= K; ++f) sp[f][oc][oslot] = predict_f(dt, f);
        }
        for (int it = 0; it < cfg.n_iter; ++it) {
            __syncthreads();   // the path is in sp; red and rq are free
            double acc[K + 1][3];
#pragma unroll
            for (int k = 0; k <= K; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[k][c] = 0.0;
            double q = 0.0;
            {
                double pi[K + 1][3];
#pragma unroll
                for (int k = 0; k <= K; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) pi[k][c] = sp[k][c][s.islot];
                for (int j = s.jb; j < s.je; ++j) {
                    double r[3], vv[3], aa[3], jj[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        r[c] = sp[0][c][j] - pi[0][c];
                        vv[c] = sp[1][c][j] - pi[1][c];
                        aa[c] = K >= 2 ? sp[K >= 2 ? 2 : 0][c][j] - pi[K >= 2 ? 2 : 0][c] : 0.0;
                        jj[c] = K >= 3 ? sp[K >= 3 ? 3 : 0][c][j] - pi[K >= 3 ? 3 : 0][c] : 0.0;
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
            }
#pragma unroll
            for (int k = 0; k <= K; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) red[k * 3 + c][s.jp * s.NI + s.islot] = acc[k][c];
            const double qw = wave_max(q);
            if (lane == 0) rq[wave] = qw;
            __syncthreads();   // the sums and maxima are in LDS; sp may change
            const bool last = it + 1 == cfg.n_iter;
            double dtn = dt;
            if (!last) {
                // the next dt from H_+ at this evaluation point (every thread
                // forms it from the same maxima)
                double qb = rq[0];
#pragma unroll
                for (int w = 1; w < kEnsWaves; ++w) qb = __builtin_fmax(qb, rq[w]);
                const double Hp = cfg.eta / sqrt(qb);
                if (!(Hp > 0.0) || !__builtin_isfinite(Hp)) {
                    failed = true;
                    break;
                }
                dtn = 0.5 * (Hm + Hp);
            }
            if (owner) {
                // a1 of this component, the j-parts added in order
                double a1[K + 1];
#pragma unroll
                for (int k = 0; k <= K; ++k) {
                    const double *rr = &red[k * 3 + oc][oslot];
                    double tsum = rr[0];
                    for (int p2 = 1; p2 < s.JP; ++p2) tsum += rr[p2 * s.NI];
                    a1[k] = tsum;
                }
                // modified corrector with this iteration's dt: velocity first, then position
                const double x0 = stl[oc][0][oslot], v0 = stl[oc][1][oslot];
                double d0[K + 1];
#pragma unroll
                for (int k = 0; k <= K; ++k) d0[k] = stl[oc][2 + k][oslot];
                double dv = 0.0;
#pragma unroll
                for (int k = P; k >= 0; --k) {
                    const double sg = (k & 1) ? (a1[k] - d0[k]) : (a1[k] + d0[k]);
                    dv = __builtin_fma(dv, dt, CV[P][k] * sg);
                }
                const double v1 = __builtin_fma(dv, dt, v0);
                double dx = 0.0;
#pragma unroll
                for (int k = P + 1; k >= 1; --k) {
                    const double sg = (k & 1) ? (a1[k - 1] - d0[k - 1]) : (a1[k - 1] + d0[k - 1]);
                    dx = __builtin_fma(dx, dt, CX[CORR][P][k] * sg);
                }
                dx = __builtin_fma(dx, dt, CX[CORR][P][0] * (v1 + v0));
                const double x1 = __builtin_fma(dx, dt, x0);
                if (!last) {
                    // the iterate, moved to t0 + dtn along its Taylor series
                    // (x1, v1, a1^(0..P)), is the next path
                    const double sh = dtn - dt;
                    double xs[P + 3];
                    xs[0] = x1;
                    xs[1] = v1;
#pragma unroll
                    for (int k = 0; k <= P; ++k) xs[k + 2] = a1[k];
#pragma unroll
                    for (int f = 0; f <= K; ++f) {
                        double acc_ = xs[P + 2];
#pragma unroll
                        for (int k = P + 1 - f; k >= 0; --k) acc_ = __builtin_fma(acc_, sh * kInvE[k + 1], xs[f + k]);
                        sp[f][oc][oslot] = acc_;
                    }
                } else {
                    // end of step: interpolated higher derivatives, the new state
                    if constexpr (P == 2) {
                        const double num = I6_A0[0] * d0[0] + I6_A1[0] * a1[0] + (I6_A0[1] * d0[1] + I6_A1[1] * a1[1]) * dt +
                                           (I6_A0[2] * d0[2] + I6_A1[2] * a1[2]) * (dt * dt);
                        stl[oc][2 + 3][oslot] = num / (dt * dt * dt);
                    }
                    if constexpr (P == 3) {
                        const double tp[4] = {1.0, dt, dt * dt, dt * dt * dt};
                        double n4 = 0.0, n5 = 0.0;
#pragma unroll
                        for (int m2 = 0; m2 <= 3; ++m2) {
                            n4 += (I8_4_A0[m2] * d0[m2] + I8_4_A1[m2] * a1[m2]) * tp[m2];
                            n5 += (I8_5_A0[m2] * d0[m2] + I8_5_A1[m2] * a1[m2]) * tp[m2];
                        }
                        stl[oc][2 + 4][oslot] = n4 / (tp[3] * dt);
                        stl[oc][2 + 5][oslot] = n5 / (tp[3] * tp[2]);
                    }
#pragma unroll
                    for (int k = 0; k <= P; ++k) stl[oc][2 + k][oslot] = a1[k];
                    stl[oc][0][oslot] = x1;
                    stl[oc][1][oslot] = v1;
                }
            }
            dt = dtn;
        }
        if (failed) break;
        t += dt;
        ++steps_here;
        // next H_- at the new positions, with the energy once past rec_from
        const bool rec = t > cfg.rec_from;
        __syncthreads();   // the new state is in LDS
        energy_and_rate(stl[0][0], stl[1][0], stl[2][0], rec, qm, E);
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
    if (olive) {
        const int64_t g = off + oslot;
        a.pos[oc * n + g] = stl[oc][0][oslot];
        a.vel[oc * n + g] = stl[oc][1][oslot];
#pragma unroll
        for (int k = 0; k < 2 * P; ++k) a.deriv[k * n3 + oc * n + g] = stl[oc][2 + k][oslot];
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
    hipLaunchKernelGGL(ens_init_kernel<1>, dim3(n_sys), dim3(kEnsInitThreads), 0, st, offsets, n, mass, path, 0, G,
                       eps2, deriv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || p < 2) return e;
    hipLaunchKernelGGL(ens_init_kernel<3>, dim3(n_sys), dim3(kEnsInitThreads), 0, st, offsets, n, mass, path, 2, G,
                       eps2, deriv + 2 * n3);
    e = hipGetLastError();
    if (e != hipSuccess || p < 3) return e;
    hipLaunchKernelGGL(ens_init_kernel<5>, dim3(n_sys), dim3(kEnsInitThreads), 0, st, offsets, n, mass, path, 4, G,
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
