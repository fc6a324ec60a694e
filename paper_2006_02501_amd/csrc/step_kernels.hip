// O(N) per-particle work of a P(EC)^n step: Taylor predictor, modified
// corrector (+ the end-of-step interpolation of the higher derivatives),
// plus the energy-diagnostic potential and a finite-value check.
//
// All of these stream FP64 SoA arrays: one lane per (component, particle)
// element of a [3][n] block, so every load and store is coalesced.
#include "hermite_coeffs.h"
#include "kernels.h"
#include "pair_chain.h"

namespace hermite {
namespace {

constexpr int kStepBlock = 256;

// 1/k for the Horner form of the Taylor series.
__device__ constexpr double kInv[9] = {0.0, 1.0, 1.0 / 2.0, 1.0 / 3.0, 1.0 / 4.0, 1.0 / 5.0, 1.0 / 6.0, 1.0 / 7.0, 1.0 / 8.0};

// Taylor predictor (Sec. 3, second paragraph) with x^(0) = x, x^(1) = v,
// x^(k+2) = a^(k), k = 0..2P-1:
//   xp = sum_{k<=2P+1} x^(k) dt^k/k!,  vp = sum_{k<=2P} x^(k+1) dt^k/k!,
//   ap = sum_{k<=2P-1} a^(k) dt^k/k!,  jp = sum_{k<=2P-2} a^(k+1) dt^k/k!.
// Evaluated in Horner form, s = c_M; s = c_k + s dt/(k+1).
// dt comes from dt_dev[0] when dt_dev is not null (a step length formed on
// the device, the variable step of Sec. 3.3).
template <int P>
__global__ __launch_bounds__(kStepBlock) void predict_kernel(int64_t n3, double dt_host,
                                                             const double *__restrict__ dt_dev,
                                                             const double *__restrict__ pos,
                                                             const double *__restrict__ vel,
                                                             const double *__restrict__ deriv,
                                                             double *__restrict__ pred)
{
    const int64_t e = (int64_t)blockIdx.x * kStepBlock + threadIdx.x;
    if (e >= n3) return;
    const double dt = dt_dev ? dt_dev[0] : dt_host;
    double xs[2 * P + 2];
    xs[0] = pos[e];
    xs[1] = vel[e];
#pragma unroll
    for (int k = 0; k < 2 * P; ++k) xs[k + 2] = deriv[(int64_t)k * n3 + e];
    // x^(first..first+M) with Taylor weights
    auto taylor = [&](int first, int M) {
        double s = xs[first + M];
#pragma unroll
        for (int k = M - 1; k >= 0; --k) s = __builtin_fma(s, dt * kInv[k + 1], xs[first + k]);
        return s;
    };
    pred[e] = taylor(0, 2 * P + 1);
    pred[n3 + e] = taylor(1, 2 * P);
    if constexpr (P >= 2) pred[2 * n3 + e] = taylor(2, 2 * P - 1);
    if constexpr (P >= 3) pred[3 * n3 + e] = taylor(3, 2 * P - 2);
}

// Modified corrector, velocity first then position (Eq. 6-8, Eq. 22-24),
// for one element; on the last iteration also the interpolated
// a^(P+1..2P-1) at the end of the step.  dt as in the predictor; a device
// dt of exactly 0 marks a step whose length could not be formed, and then
// nothing is written.
// With comp ([2][3][n], x then v) the increments dt*dv and dt*dx are added
// by Kahan's compensated summation (the option of Sec. 3.2): y = inc - c,
// s' = s + y, c' = (s' - s) - y.  Every iterate uses the carried c; the last
// iteration stores c'.
// Before the last iteration the iterate becomes the next path: (x1, v1) and
// the evaluated a, adot.  In a variable step (dtn_dev not null) the next
// iteration's step length dtn differs from this one's, and the path is the
// iterate moved to the new end point along its own Taylor series,
// x^(f) + sum_k x^(f+k) d^k/k! with x^(0..P+2) = (x1, v1, a1^(0..P)) and
// d = dtn - dt (Horner form, as the predictor).
template <int P, int CORR>
__global__ __launch_bounds__(kStepBlock) void correct_kernel(int64_t n3, double dt_host,
                                                             const double *__restrict__ dt_dev,
                                                             const double *__restrict__ dtn_dev, int last,
                                                             double *__restrict__ pos,
                                                             double *__restrict__ vel, double *__restrict__ deriv,
                                                             const double *__restrict__ eval,
                                                             double *__restrict__ pred, double *__restrict__ comp)
{
    const int64_t e = (int64_t)blockIdx.x * kStepBlock + threadIdx.x;
    const double dt = dt_dev ? dt_dev[0] : dt_host;
    if (e >= n3 || dt == 0.0) return;
    double a0[P + 1], a1[P + 1];
#pragma unroll
    for (int k = 0; k <= P; ++k) {
        a0[k] = deriv[(int64_t)k * n3 + e];
        a1[k] = eval[(int64_t)k * n3 + e];
    }
    const double x0 = pos[e], v0 = vel[e];
    // v1 - v0 = dt (c0 s0 + dt (c1 s1 + dt (c2 s2 + ...)))
    double dv = 0.0;
#pragma unroll
    for (int k = P; k >= 0; --k) {
        const double s = (k & 1) ? (a1[k] - a0[k]) : (a1[k] + a0[k]);
        dv = __builtin_fma(dv, dt, CV[P][k] * s);
    }
    double v1, cv1 = 0.0;
    if (comp) {
        const double y = dv * dt - comp[n3 + e];
        v1 = v0 + y;
        cv1 = (v1 - v0) - y;
    } else {
        v1 = __builtin_fma(dv, dt, v0);
    }
    // q^(0) = v, q^(k) = a^(k-1)
    double dx = 0.0;
#pragma unroll
    for (int k = P + 1; k >= 1; --k) {
        const double s = (k & 1) ? (a1[k - 1] - a0[k - 1]) : (a1[k - 1] + a0[k - 1]);
        dx = __builtin_fma(dx, dt, CX[CORR][P][k] * s);
    }
    dx = __builtin_fma(dx, dt, CX[CORR][P][0] * (v1 + v0));
    double x1, cx1 = 0.0;
    if (comp) {
        const double y = dx * dt - comp[e];
        x1 = x0 + y;
        cx1 = (x1 - x0) - y;
    } else {
        x1 = __builtin_fma(dx, dt, x0);
    }
    if (!last) {
        if (dtn_dev) {
            const double d = dtn_dev[0] - dt;
            double xs[P + 3];
            xs[0] = x1;
            xs[1] = v1;
#pragma unroll
            for (int k = 0; k <= P; ++k) xs[k + 2] = a1[k];
#pragma unroll
            for (int f = 0; f <= P; ++f) {
                double t = xs[P + 2];
#pragma unroll
                for (int k = P + 1 - f; k >= 0; --k) t = __builtin_fma(t, d * kInv[k + 1], xs[f + k]);
                pred[(int64_t)f * n3 + e] = t;
            }
            return;
        }
        // next iterate: (x1, v1) and the evaluated a, adot as the relative path
        pred[e] = x1;
        pred[n3 + e] = v1;
#pragma unroll
        for (int m = 0; m <= P - 2; ++m) pred[(int64_t)(2 + m) * n3 + e] = a1[m];
        return;
    }
    pos[e] = x1;
    vel[e] = v1;
    if (comp) {
        comp[e] = cx1;
        comp[n3 + e] = cv1;
    }
    if constexpr (P == 2) {
        const double t1 = dt, t2 = dt * dt;
        const double num = I6_A0[0] * a0[0] + I6_A1[0] * a1[0] + (I6_A0[1] * a0[1] + I6_A1[1] * a1[1]) * t1 +
                           (I6_A0[2] * a0[2] + I6_A1[2] * a1[2]) * t2;
        deriv[3 * n3 + e] = num / (t2 * dt);
    }
    if constexpr (P == 3) {
        const double t1 = dt, t2 = dt * dt, t3 = t2 * dt;
        double n4 = 0.0, n5 = 0.0;
        const double tp[4] = {1.0, t1, t2, t3};
#pragma unroll
        for (int m = 0; m <= 3; ++m) {
            n4 += (I8_4_A0[m] * a0[m] + I8_4_A1[m] * a1[m]) * tp[m];
            n5 += (I8_5_A0[m] * a0[m] + I8_5_A1[m] * a1[m]) * tp[m];
        }
        deriv[4 * n3 + e] = n4 / (t3 * dt);
        deriv[5 * n3 + e] = n5 / (t3 * t2);
    }
#pragma unroll
    for (int k = 0; k <= P; ++k) deriv[(int64_t)k * n3 + e] = a1[k];
}

__global__ __launch_bounds__(kStepBlock) void potential_kernel(int64_t n, const double *__restrict__ mass,
                                                               const double *__restrict__ pos, double G, double eps2,
                                                               double *__restrict__ phi)
{
    __shared__ double tile[kStepBlock * 4];
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kStepBlock + tid;
    const bool ok = i < n;
    const double xi = ok ? pos[i] : 0.0, yi = ok ? pos[n + i] : 0.0, zi = ok ? pos[2 * n + i] : 0.0;
    double s = 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += kStepBlock) {
        const int cnt = (int)min((int64_t)kStepBlock, n - j0);
        __syncthreads();
        if (tid < cnt) {
            tile[4 * tid + 0] = G * mass[j0 + tid];
            tile[4 * tid + 1] = pos[j0 + tid];
            tile[4 * tid + 2] = pos[n + j0 + tid];
            tile[4 * tid + 3] = pos[2 * n + j0 + tid];
        }
        __syncthreads();
        for (int jj = 0; jj < cnt; ++jj) {
            const double dx = tile[4 * jj + 1] - xi, dy = tile[4 * jj + 2] - yi, dz = tile[4 * jj + 3] - zi;
            double w = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
            const bool self = (j0 + jj == i);
            w = self ? 1.0 : w;
            const double m = self ? 0.0 : tile[4 * jj];
            s = __builtin_fma(-m, rsqrt64(w), s);
        }
    }
    if (ok) phi[i] = s;
}

__global__ __launch_bounds__(kStepBlock) void check_finite_kernel(const double *__restrict__ a, int64_t count,
                                                                  int *__restrict__ flag)
{
    int bad = 0;
    for (int64_t e = (int64_t)blockIdx.x * kStepBlock + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * kStepBlock) {
        bad |= __builtin_isfinite(a[e]) ? 0 : 1;
    }
    if (bad) flag[0] = 1;
}

inline unsigned blocks_for(int64_t count) { return (unsigned)((count + kStepBlock - 1) / kStepBlock); }

template <int P>
hipError_t correct_p(int corrector, int last, int64_t n3, double dt, const double *dt_dev, const double *dtn_dev,
                     double *pos, double *vel, double *deriv, const double *eval, double *pred, double *comp,
                     hipStream_t st)
{
    const dim3 g(blocks_for(n3)), b(kStepBlock);
    switch (corrector) {
        case 0: hipLaunchKernelGGL((correct_kernel<P, 0>), g, b, 0, st, n3, dt, dt_dev, dtn_dev, last, pos, vel, deriv, eval, pred, comp); break;
        case 1: hipLaunchKernelGGL((correct_kernel<P, 1>), g, b, 0, st, n3, dt, dt_dev, dtn_dev, last, pos, vel, deriv, eval, pred, comp); break;
        case 2: hipLaunchKernelGGL((correct_kernel<P, 2>), g, b, 0, st, n3, dt, dt_dev, dtn_dev, last, pos, vel, deriv, eval, pred, comp); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_predict(int p, int64_t n, double dt, const double *dt_dev, const double *pos, const double *vel,
                          const double *deriv, double *pred, hipStream_t st)
{
    const int64_t n3 = 3 * n;
    if (n3 <= 0) return hipSuccess;
    const dim3 g(blocks_for(n3)), b(kStepBlock);
    switch (p) {
        case 1: hipLaunchKernelGGL(predict_kernel<1>, g, b, 0, st, n3, dt, dt_dev, pos, vel, deriv, pred); break;
        case 2: hipLaunchKernelGGL(predict_kernel<2>, g, b, 0, st, n3, dt, dt_dev, pos, vel, deriv, pred); break;
        case 3: hipLaunchKernelGGL(predict_kernel<3>, g, b, 0, st, n3, dt, dt_dev, pos, vel, deriv, pred); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_correct(int p, int corrector, int last, int64_t n, double dt, const double *dt_dev,
                          const double *dtn_dev, double *pos, double *vel, double *deriv, const double *eval,
                          double *pred, double *comp, hipStream_t st)
{
    const int64_t n3 = 3 * n;
    if (n3 <= 0) return hipSuccess;
    switch (p) {
        case 1: return correct_p<1>(corrector, last, n3, dt, dt_dev, dtn_dev, pos, vel, deriv, eval, pred, comp, st);
        case 2: return correct_p<2>(corrector, last, n3, dt, dt_dev, dtn_dev, pos, vel, deriv, eval, pred, comp, st);
        case 3: return correct_p<3>(corrector, last, n3, dt, dt_dev, dtn_dev, pos, vel, deriv, eval, pred, comp, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_potential(int64_t n, const double *mass, const double *pos, double G, double eps2, double *phi,
                            hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(potential_kernel, dim3(blocks_for(n)), dim3(kStepBlock), 0, st, n, mass, pos, G, eps2, phi);
    return hipGetLastError();
}

hipError_t launch_check_finite(const double *data, int64_t count, int *flag, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = blocks_for(count);
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)blocks), dim3(kStepBlock), 0, st, data, count, flag);
    return hipGetLastError();
}

}  // namespace hermite
