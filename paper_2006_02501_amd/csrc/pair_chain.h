// Per-pair time derivatives of the softened acceleration
//     A(t) = G m_j r(t) w(t)^(-3/2),   w = r.r + eps^2,   r = x_j - x_i
// (force law of the paper's Sec. 3), with the relative path r, v = r', a = r'',
// j = r''' taken from the particles' x, v, a, adot.
//
// Derivation used here (normalised derivatives of w^(3/2)): with
// g = w^(3/2), r = g A / (G m_j), so Leibniz on r^(n) = (g A)^(n) / (G m_j)
// gives
//     A^(n) = mu r^(n) - sum_{k=1..n} C(n,k) G_k A^(n-k),   mu = G m_j / g,
// where G_k = g^(k)/g follows from w g' = (3/2) w' g:
//     G_0 = 1,
//     G_{n+1} = (3/2) sum_{k=0..n} C(n,k) W_{k+1} G_{n-k} - sum_{k=1..n} C(n,k) W_k G_{n+1-k},
//     W_k = w^(k)/w,  w^(k) = sum_l C(k,l) r^(l).r^(k-l)   (k >= 1).
// For k <= 3 this is the familiar chain (alpha = G_1/3, beta = G_2/3,
// gamma = G_3/3):
//     alpha = r.v/w,  beta = (v.v + r.a)/w + alpha^2,
//     gamma = (3 v.a + r.j)/w + alpha (3 beta - 4 alpha^2),
//     A = mu r,  J = mu v - 3 alpha A,  S = mu a - 6 alpha J - 3 beta A,
//     C = mu j - 9 alpha S - 9 beta J - 3 gamma A.
// The hot path factors mu out (A = mu r', J = mu J', ...) so every
// accumulation is one fused multiply-add.
#pragma once

#include <hip/hip_runtime.h>

namespace hermite {

// 1/sqrt(w) in FP64: the hardware estimate refined by one third-order
// Newton-type step, y' = y (1 + e/2 + 3 e^2/8), e = 1 - w y^2 (error ~ e^3).
__device__ __forceinline__ double rsqrt64(double w)
{
    const double y = __builtin_amdgcn_rsq(w);
    const double e = __builtin_fma(-w, y * y, 1.0);
    const double t = __builtin_fma(e, 0.375, 0.5);
    return __builtin_fma(y * e, t, y);
}

__device__ __forceinline__ float rsqrt32(float w) { return __builtin_amdgcn_rsqf(w); }

__device__ __forceinline__ double rsqrt_t(double w) { return rsqrt64(w); }
__device__ __forceinline__ float rsqrt_t(float w) { return rsqrt32(w); }

// Fused multiply-add in the operands' own precision (the plain builtin is the
// double one and would silently promote a float chain).
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// One pair, derivatives 0..K (K <= 3), relative path components given.
// mr3 = G m_j w^(-3/2), rinv2 = 1/w.  Adds mr3 * (r, J', S', C') into acc.
// The chain's coefficients are formed already negated (n1 = -3 alpha, ...),
// so every vector update is a plain fused multiply-add onto a value that is
// not needed afterwards: on gfx950 these take the two-operand accumulate
// encoding (v_fmac), which issues at a higher rate than the three-operand form.
template <int K, typename T>
__device__ __forceinline__ void chain_accumulate(const T (&r)[3], const T (&v)[3], const T (&a)[3],
                                                 const T (&j)[3], T mr3, T rinv2, T (&acc)[K + 1][3])
{
    static_assert(K >= 1 && K <= 3, "chain supports 1..3 derivatives");
    const T rv = fma_t(r[2], v[2], fma_t(r[1], v[1], r[0] * v[0]));
    const T alpha = rv * rinv2;
    T vv = T(0), ra = T(0), va = T(0), rj = T(0);
    if constexpr (K >= 2) {
        vv = fma_t(v[2], v[2], fma_t(v[1], v[1], v[0] * v[0]));
        ra = fma_t(r[2], a[2], fma_t(r[1], a[1], r[0] * a[0]));
    }
    if constexpr (K >= 3) {
        va = fma_t(v[2], a[2], fma_t(v[1], a[1], v[0] * a[0]));
        rj = fma_t(r[2], j[2], fma_t(r[1], j[1], r[0] * j[0]));
    }
    const T n1 = T(-3) * alpha;                  // -3 alpha
    T J[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc[0][c] = fma_t(mr3, r[c], acc[0][c]);
        J[c] = fma_t(n1, r[c], v[c]);
        acc[1][c] = fma_t(mr3, J[c], acc[1][c]);
    }
    if constexpr (K >= 2) {
        const T alpha2 = alpha * alpha;
        const T beta = fma_t(vv + ra, rinv2, alpha2);
        const T n2 = T(2) * n1;                  // -6 alpha
        const T n3 = T(-3) * beta;               // -3 beta
        T S[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            S[c] = fma_t(n3, r[c], fma_t(n2, J[c], a[c]));
            acc[2][c] = fma_t(mr3, S[c], acc[2][c]);
        }
        if constexpr (K >= 3) {
            // gamma = (3 v.a + r.j)/w + alpha (3 beta - 4 alpha^2)
            const T gamma = fma_t(fma_t(T(3), va, rj), rinv2, alpha * fma_t(T(-4), alpha2, T(-1) * n3));
            const T n4 = T(3) * n1;              // -9 alpha
            const T n5 = T(3) * n3;              // -9 beta
            const T n6 = T(-3) * gamma;          // -3 gamma
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T C = fma_t(n6, r[c], fma_t(n5, J[c], fma_t(n4, S[c], j[c])));
                acc[3][c] = fma_t(mr3, C, acc[3][c]);
            }
        }
    }
}

// One pair taken once for both of its bodies: the chain's vectors
// (r, J', S', C') are odd under the exchange of i and j (every relative path
// derivative changes sign, alpha, beta and gamma do not), so body i adds
// G m_j w^(-3/2) times them and body j adds -G m_i w^(-3/2) times them.
// mj3 = G m_j w^(-3/2), nmi3 = -G m_i w^(-3/2), rinv2 = 1/w; T is double
// (FP64 chain) or float (mixed chain, from the FP64 differences' casts).
template <int K, typename T>
__device__ __forceinline__ void chain_pair(const T (&r)[3], const T (&v)[3], const T (&a)[3], const T (&j)[3],
                                           T mj3, T nmi3, T rinv2, T (&acc_i)[K + 1][3], T (&acc_j)[K + 1][3])
{
    static_assert(K >= 1 && K <= 3, "chain supports 1..3 derivatives");
    const T rv = fma_t(r[2], v[2], fma_t(r[1], v[1], r[0] * v[0]));
    const T alpha = rv * rinv2;
    T vv = T(0), ra = T(0), va = T(0), rj = T(0);
    if constexpr (K >= 2) {
        vv = fma_t(v[2], v[2], fma_t(v[1], v[1], v[0] * v[0]));
        ra = fma_t(r[2], a[2], fma_t(r[1], a[1], r[0] * a[0]));
    }
    if constexpr (K >= 3) {
        va = fma_t(v[2], a[2], fma_t(v[1], a[1], v[0] * a[0]));
        rj = fma_t(r[2], j[2], fma_t(r[1], j[1], r[0] * j[0]));
    }
    const T n1 = T(-3) * alpha;
    T J[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc_i[0][c] = fma_t(mj3, r[c], acc_i[0][c]);
        acc_j[0][c] = fma_t(nmi3, r[c], acc_j[0][c]);
        J[c] = fma_t(n1, r[c], v[c]);
        acc_i[1][c] = fma_t(mj3, J[c], acc_i[1][c]);
        acc_j[1][c] = fma_t(nmi3, J[c], acc_j[1][c]);
    }
    if constexpr (K >= 2) {
        const T alpha2 = alpha * alpha;
        const T beta = fma_t(vv + ra, rinv2, alpha2);
        const T n2 = T(2) * n1;
        const T n3 = T(-3) * beta;
        T S[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            S[c] = fma_t(n3, r[c], fma_t(n2, J[c], a[c]));
            acc_i[2][c] = fma_t(mj3, S[c], acc_i[2][c]);
            acc_j[2][c] = fma_t(nmi3, S[c], acc_j[2][c]);
        }
        if constexpr (K >= 3) {
            const T gamma = fma_t(fma_t(T(3), va, rj), rinv2, alpha * fma_t(T(-4), alpha2, T(-1) * n3));
            const T n4 = T(3) * n1;
            const T n5 = T(3) * n3;
            const T n6 = T(-3) * gamma;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T C = fma_t(n6, r[c], fma_t(n5, J[c], fma_t(n4, S[c], j[c])));
                acc_i[3][c] = fma_t(mj3, C, acc_i[3][c]);
                acc_j[3][c] = fma_t(nmi3, C, acc_j[3][c]);
            }
        }
    }
}

// The split chain taken once for both bodies: orders 0 and 1 in FP64 with
// exactly chain_pair<K, double>'s operations (so the same bits), orders 2..K
// in FP32 as chain_split forms them, each body with its own mass factor.
template <int K>
__device__ __forceinline__ void chain_split_pair(const double (&r)[3], const double (&v)[3], const float (&af)[3],
                                                 const float (&jf)[3], double mj3, double nmi3, double rinv2,
                                                 double (&acc_i)[K + 1][3], double (&acc_j)[K + 1][3],
                                                 float (&accf_i)[K + 1][3], float (&accf_j)[K + 1][3])
{
    static_assert(K >= 2 && K <= 3, "the split chain has FP32 orders 2..K");
    const double rv = fma_t(r[2], v[2], fma_t(r[1], v[1], r[0] * v[0]));
    const double alpha = rv * rinv2;
    const double n1 = -3.0 * alpha;
    float Jf[3], rf[3], vf[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc_i[0][c] = fma_t(mj3, r[c], acc_i[0][c]);
        acc_j[0][c] = fma_t(nmi3, r[c], acc_j[0][c]);
        const double J = fma_t(n1, r[c], v[c]);
        acc_i[1][c] = fma_t(mj3, J, acc_i[1][c]);
        acc_j[1][c] = fma_t(nmi3, J, acc_j[1][c]);
        Jf[c] = (float)J;
        rf[c] = (float)r[c];
        vf[c] = (float)v[c];
    }
    const float alf = (float)alpha, r2f = (float)rinv2, mfi = (float)mj3, mfj = (float)nmi3;
    const float vv = fma_t(vf[2], vf[2], fma_t(vf[1], vf[1], vf[0] * vf[0]));
    const float ra = fma_t(rf[2], af[2], fma_t(rf[1], af[1], rf[0] * af[0]));
    const float alpha2 = alf * alf;
    const float beta = fma_t(vv + ra, r2f, alpha2);
    const float n1f = -3.0f * alf;
    const float n2 = 2.0f * n1f;
    const float n3 = -3.0f * beta;
    float S[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        S[c] = fma_t(n3, rf[c], fma_t(n2, Jf[c], af[c]));
        accf_i[2][c] = fma_t(mfi, S[c], accf_i[2][c]);
        accf_j[2][c] = fma_t(mfj, S[c], accf_j[2][c]);
    }
    if constexpr (K >= 3) {
        const float va = fma_t(vf[2], af[2], fma_t(vf[1], af[1], vf[0] * af[0]));
        const float rj = fma_t(rf[2], jf[2], fma_t(rf[1], jf[1], rf[0] * jf[0]));
        const float gamma = fma_t(fma_t(3.0f, va, rj), r2f, alf * fma_t(-4.0f, alpha2, -1.0f * n3));
        const float n4 = 3.0f * n1f;
        const float n5 = 3.0f * n3;
        const float n6 = -3.0f * gamma;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float C = fma_t(n6, rf[c], fma_t(n5, Jf[c], fma_t(n4, S[c], jf[c])));
            accf_i[3][c] = fma_t(mfi, C, accf_i[3][c]);
            accf_j[3][c] = fma_t(mfj, C, accf_j[3][c]);
        }
    }
}

// Split precision (Sec. 4: lower precision for the higher derivatives only):
// a and adot exactly as chain_accumulate<K, double> forms them (the same
// operations, so the same bits), a^(2) and a^(3) in FP32 from the FP32 casts
// of the relative path and of alpha, J' and the FP64 factors.
template <int K>
__device__ __forceinline__ void chain_split(const double (&r)[3], const double (&v)[3], const float (&af)[3],
                                            const float (&jf)[3], double mr3, double rinv2, double (&acc)[K + 1][3],
                                            float (&accf)[K + 1][3])
{
    static_assert(K >= 2 && K <= 3, "the split chain has FP32 orders 2..K");
    const double rv = fma_t(r[2], v[2], fma_t(r[1], v[1], r[0] * v[0]));
    const double alpha = rv * rinv2;
    const double n1 = -3.0 * alpha;
    float Jf[3], rf[3], vf[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc[0][c] = fma_t(mr3, r[c], acc[0][c]);
        const double J = fma_t(n1, r[c], v[c]);
        acc[1][c] = fma_t(mr3, J, acc[1][c]);
        Jf[c] = (float)J;
        rf[c] = (float)r[c];
        vf[c] = (float)v[c];
    }
    const float alf = (float)alpha, r2f = (float)rinv2, mf = (float)mr3;
    const float vv = fma_t(vf[2], vf[2], fma_t(vf[1], vf[1], vf[0] * vf[0]));
    const float ra = fma_t(rf[2], af[2], fma_t(rf[1], af[1], rf[0] * af[0]));
    const float alpha2 = alf * alf;
    const float beta = fma_t(vv + ra, r2f, alpha2);
    const float n1f = -3.0f * alf;
    const float n2 = 2.0f * n1f;                 // -6 alpha
    const float n3 = -3.0f * beta;               // -3 beta
    float S[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        S[c] = fma_t(n3, rf[c], fma_t(n2, Jf[c], af[c]));
        accf[2][c] = fma_t(mf, S[c], accf[2][c]);
    }
    if constexpr (K >= 3) {
        const float va = fma_t(vf[2], af[2], fma_t(vf[1], af[1], vf[0] * af[0]));
        const float rj = fma_t(rf[2], jf[2], fma_t(rf[1], jf[1], rf[0] * jf[0]));
        const float gamma = fma_t(fma_t(3.0f, va, rj), r2f, alf * fma_t(-4.0f, alpha2, -1.0f * n3));
        const float n4 = 3.0f * n1f;             // -9 alpha
        const float n5 = 3.0f * n3;              // -9 beta
        const float n6 = -3.0f * gamma;          // -3 gamma
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float C = fma_t(n6, rf[c], fma_t(n5, Jf[c], fma_t(n4, S[c], jf[c])));
            accf[3][c] = fma_t(mf, C, accf[3][c]);
        }
    }
}

// Binomial coefficient (compile time).
__host__ __device__ constexpr double binom(int n, int k)
{
    double c = 1.0;
    for (int i = 1; i <= k; ++i) c = c * double(n - k + i) / double(i);
    return c;
}

// Generic order K <= 5 (FP64), used by the explicit-derivative
// initialisation: r[k] = k-th derivative of the relative path.
template <int K>
__device__ __forceinline__ void generic_accumulate(const double (&r)[K + 1][3], double eps2, double gm,
                                                   bool zero, double (&acc)[K + 1][3])
{
    double w0 = __builtin_fma(r[0][0], r[0][0], __builtin_fma(r[0][1], r[0][1], __builtin_fma(r[0][2], r[0][2], eps2)));
    if (zero) w0 = 1.0;
    const double rinv = rsqrt64(w0);
    const double rinv2 = rinv * rinv;
    const double mu = zero ? 0.0 : gm * rinv * rinv2;
    double W[K + 1];
    W[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= K; ++k) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l <= k; ++l)
            s += binom(k, l) * (r[l][0] * r[k - l][0] + r[l][1] * r[k - l][1] + r[l][2] * r[k - l][2]);
        W[k] = s * rinv2;
    }
    double Gk[K + 1];
    Gk[0] = 1.0;
#pragma unroll
    for (int m = 0; m < K; ++m) {
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int k = 0; k <= m; ++k) s1 += binom(m, k) * W[k + 1] * Gk[m - k];
#pragma unroll
        for (int k = 1; k <= m; ++k) s2 += binom(m, k) * W[k] * Gk[m + 1 - k];
        Gk[m + 1] = 1.5 * s1 - s2;
    }
    double A[K + 1][3];
#pragma unroll
    for (int m = 0; m <= K; ++m) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double s = mu * r[m][c];
#pragma unroll
            for (int k = 1; k <= m; ++k) s -= binom(m, k) * Gk[k] * A[m - k][c];
            A[m][c] = s;
            acc[m][c] += s;
        }
    }
}

}  // namespace hermite
