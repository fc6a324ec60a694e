// Variable, time-symmetric step of Sec. 3.3 (Eq. 25).
//
// The criterion is the shortest two-body Kepler time scale over all pairs,
//     H(x) = eta min_{i != j} ((r_ij^2 + eps^2)^(3/2) / (G (m_i + m_j)))^(1/2)
//          = eta q^(-1/2),   q = max_{i != j} G (m_i + m_j) (r_ij^2 + eps^2)^(-3/2),
// and the step it gives is kept on the device so that a step never waits on
// the host between its launches: the prediction uses s H(x0) and the
// correction after the evaluation at the iterate x_k uses
// s (H(x0) + H(x_k)) / 2, with s = +1 or -1 the direction of integration.
//
// q is a max over the N (N - 1) / 2 unordered pairs (the rate is symmetric in
// i and j, and so is the way it is rounded here): ~20 FP64 VALU operations
// per pair (difference, softened distance, refined reciprocal square root,
// its cube, the mass sum, the max), against ~90 per pair of the 8th-order
// evaluation.  Workgroups cover (256 i-particles) x (a j-range) and take the
// pairs with j > i; each writes one maximum (0 when it holds no such pair),
// and a single-workgroup kernel folds them and forms H and dt.  A maximum
// does not depend on the order it is taken in, so the result is the same for
// every launch shape.
#include "kernels.h"
#include "pair_chain.h"

namespace hermite {
namespace {

constexpr int kQBlock = 256;
constexpr int kQWaves = kQBlock / 64;

// Larger rate of two (v_max_f64: a NaN operand is dropped, so a pair with
// a non-finite position does not set the step; the finite-value check of the
// state reports such positions).
__device__ __forceinline__ double qcombine(double a, double b) { return __builtin_fmax(a, b); }

__device__ __forceinline__ double wave_qmax(double q)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) q = qcombine(q, __shfl_xor(q, off, 64));
    return q;
}

__device__ __forceinline__ double block_qmax(double q)
{
    __shared__ double red[kQWaves];
    q = wave_qmax(q);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = q;
    __syncthreads();
    q = red[0];
#pragma unroll
    for (int w = 1; w < kQWaves; ++w) q = qcombine(red[w], q);
    return q;
}

// qpart[blockIdx.y * gridDim.x + blockIdx.x] = max of the rate over
// i in this workgroup's 256 and j in [blockIdx.y * j_chunk, +j_chunk), j > i.
// The j loop index is uniform, so the j-particle loads go through the scalar
// unit; each lane keeps its own i.
__global__ __launch_bounds__(kQBlock) void qmax_kernel(int64_t n, const double *__restrict__ mass,
                                                       const double *__restrict__ x, double G, double eps2,
                                                       int64_t j_chunk, double *__restrict__ qpart)
{
    const int64_t ib0 = (int64_t)blockIdx.x * kQBlock;
    const int64_t i = ib0 + threadIdx.x;
    const bool live = i < n;
    const int64_t ic = live ? i : n - 1;
    const double xi = x[ic], yi = x[n + ic], zi = x[2 * n + ic];
    const double mi = mass[ic];
    // pairs with j > i only: no j at or below the block's first i
    const int64_t j0 = max((int64_t)blockIdx.y * j_chunk, ib0 + 1);
    const int64_t j1 = min((int64_t)blockIdx.y * j_chunk + j_chunk, n);
    double best = 0.0;
    // the rate of pair (i, j); a larger finite rate replaces best (a NaN rate
    // compares false and is dropped, as qcombine drops it)
    auto rate = [&](int64_t j) {
        const double dx = x[j] - xi, dy = x[n + j] - yi, dz = x[2 * n + j] - zi;
        const double mj = mass[j];
        const double w = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
        const double y = rsqrt64(w);
        return (G * (mj + mi)) * (y * y * y);
    };
    if (j0 >= ib0 + kQBlock) {
        // every j of the range lies above every i of the workgroup
#pragma unroll 4
        for (int64_t j = j0; j < j1; ++j) {
            const double q = rate(j);
            best = q > best ? q : best;
        }
    } else {
        // the range meets the workgroup's own i: the pairs with j <= i (taken
        // from their other end, or the self pair, whose rate may be inf or
        // NaN without softening) are left out by the select; every load of j
        // is unconditional (a uniform scalar load)
#pragma unroll 4
        for (int64_t j = j0; j < j1; ++j) {
            const double q = rate(j);
            best = (j > i && q > best) ? q : best;
        }
    }
    best = block_qmax(live ? best : 0.0);
    if (threadIdx.x == 0) qpart[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = best;
}

// vs[0] = H_- (start of step), vs[2] = latest H_+, vs[3] = 1 once the
// criterion is undefined (q not positive and finite: no massive pair,
// coincident unsoftened bodies, or no finite position at all); vs[slot] (1 or
// 4) receives a step length.  mode 0 starts a step (H_- and dt = s H_-,
// clears vs[3]); mode 1 takes H_+ at an end point (dt = s (H_- + H_+)/2).
// Once vs[3] is set the dt written is 0, which the predictor and the
// corrector take as "leave the state as it is".
__global__ __launch_bounds__(kQBlock) void timestep_kernel(const double *__restrict__ qpart, int count, double eta,
                                                           double dir, int mode, int slot,
                                                           double *__restrict__ vs)
{
    double q = 0.0;
    for (int k = threadIdx.x; k < count; k += kQBlock) q = qcombine(qpart[k], q);
    q = block_qmax(q);
    if (threadIdx.x != 0) return;
    const double H = eta / sqrt(q);
    const bool bad = !(q > 0.0) || !__builtin_isfinite(H) || !(H > 0.0);
    const bool failed = bad || (mode == 1 && vs[3] != 0.0);
    double dt;
    if (mode == 0) {
        vs[0] = H;
        dt = dir * H;
    } else {
        vs[2] = H;
        dt = dir * (0.5 * (vs[0] + H));
    }
    vs[slot] = failed ? 0.0 : dt;
    vs[3] = failed ? 1.0 : 0.0;
}

}  // namespace

int qmax_partials(int64_t n, int *nsplit_out, int64_t *j_chunk_out)
{
    const int64_t nib = (n + kQBlock - 1) / kQBlock;
    // about 8192 workgroups when N allows it (half of them hold no pair with
    // j > i), each j-range at least 128 long (at 131k bodies 11 % faster than
    // 4096 workgroups of at least 256; the same at 16k)
    int64_t ns = (8192 + nib - 1) / nib;
    const int64_t max_ns = (n + 127) / 128;
    if (ns > max_ns) ns = max_ns;
    if (ns < 1) ns = 1;
    const int64_t chunk = (n + ns - 1) / ns;
    ns = (n + chunk - 1) / chunk;
    if (nsplit_out) *nsplit_out = (int)ns;
    if (j_chunk_out) *j_chunk_out = chunk;
    return (int)(nib * ns);
}

hipError_t launch_timestep(int64_t n, const double *mass, const double *x, double G, double eps2, double eta,
                           double dir, int mode, int slot, double *qpart, int64_t qpart_cap, double *vs,
                           hipStream_t st)
{
    if (n < 2 || (slot != 1 && slot != 4)) return hipErrorInvalidValue;
    int ns = 1;
    int64_t chunk = n;
    const int count = qmax_partials(n, &ns, &chunk);
    if (count > qpart_cap) return hipErrorInvalidValue;
    const unsigned nib = (unsigned)((n + kQBlock - 1) / kQBlock);
    hipLaunchKernelGGL(qmax_kernel, dim3(nib, (unsigned)ns), dim3(kQBlock), 0, st, n, mass, x, G, eps2, chunk, qpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(timestep_kernel, dim3(1), dim3(kQBlock), 0, st, qpart, count, eta, dir, mode, slot, vs);
    return hipGetLastError();
}

hipError_t launch_timestep_fold(const double *qpart, int count, double eta, double dir, int mode, int slot,
                                double *vs, hipStream_t st)
{
    if (count < 1 || (slot != 1 && slot != 4)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(timestep_kernel, dim3(1), dim3(kQBlock), 0, st, qpart, count, eta, dir, mode, slot, vs);
    return hipGetLastError();
}

}  // namespace hermite
