/*
 * ORACLE -- test infrastructure only.  Nothing in the product path may link,
 * load or call this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark do.
 *
 * Plain FP64 direct summation of the softened pair acceleration used by the
 * paper's numerical tests (Sec. 3 opening paragraph):
 *
 *     a_ij = G m_j r_ij (r_ij^2 + eps^2)^(-3/2),      r_ij = x_j - x_i,
 *
 * and of its first K time derivatives along a particle path whose time
 * derivatives x^(0..K) are given (x, v, a, adot, ...).  The order-2(p+1)
 * integrator needs K = p derivatives per evaluation (Sec. 2, after Eq. 8), and
 * the explicit-derivative initialisation needs up to the 5th (Sec. 3, second
 * paragraph).
 *
 * Method: the definition written out with the product rule (Leibniz).
 *   w(t)   = r.r + eps^2,       w^(n) = sum_l C(n,l) r^(l).r^(n-l)
 *   u(t)   = w^(-3/2),          from w u' = -(3/2) w' u differentiated n times:
 *            w u^(n+1) = -(3/2) sum_{k=0..n} C(n,k) w^(k+1) u^(n-k)
 *                        -      sum_{k=1..n} C(n,k) w^(k)   u^(n-k+1)
 *   a^(n)  = G m_j sum_k C(n,k) r^(k) u^(n-k)
 * The sum over j runs in index order, j != i (self term excluded by index).
 * Compile with -ffp-contract=off: no fused multiply-adds, IEEE rounding.
 *
 * Also: per-i potential  phi_i = -sum_{j != i} G m_j (r_ij^2 + eps^2)^(-1/2),
 * the potential whose gradient is the force above (energy diagnostic of
 * Sec. 3.1).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_KMAX 5

static double binom(int n, int k)
{
    double c = 1.0;
    for (int i = 1; i <= k; ++i) c = c * (double)(n - k + i) / (double)i;
    return c;
}

/*
 * n        number of particles
 * mass     [n]
 * path     [(K+1)][3][n]   path[(k*3+c)*n + idx] = d^k x_c / dt^k of particle idx
 * K        highest derivative wanted, 0..5
 * n_i      number of target particles; i_list[n_i] their indices (NULL = all, n_i = n)
 * out      [(K+1)][3][n_i] result a^(k)_c for each target
 * mag      [(K+1)][n_i]    sum over j of |a_ij^(k)| (Euclidean), may be NULL
 * nat      [(K+1)][n_i]    sum over j of the pair's natural k-th derivative scale
 *                          G m_j s^-2 omega^k, s = sqrt(r.r + eps^2), omega the
 *                          fastest rate of the relative path, max_k (|r^(k)|/s)^(1/k):
 *                          the size of the change that a relative rounding of
 *                          r, v, a, ... produces in a^(k).  May be NULL.
 * returns 0 on success, -1 on bad arguments, -2 if any output is not finite
 */
int oracle_pair_derivs(int64_t n, const double *mass, const double *path, int32_t K,
                       double G, double eps2, int64_t n_i, const int64_t *i_list,
                       double *out, double *mag, double *nat)
{
    if (n < 0 || K < 0 || K > ORACLE_KMAX || eps2 < 0.0 || !mass || !path || !out) return -1;
    if (!i_list) n_i = n;
    if (n_i < 0) return -1;
    double C[ORACLE_KMAX + 1][ORACLE_KMAX + 1];
    for (int a = 0; a <= ORACLE_KMAX; ++a)
        for (int b = 0; b <= ORACLE_KMAX; ++b) C[a][b] = (b <= a) ? binom(a, b) : 0.0;

    int bad = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(| : bad)
    for (int64_t ii = 0; ii < n_i; ++ii) {
        const int64_t i = i_list ? i_list[ii] : ii;
        if (i < 0 || i >= n) { bad |= 1; continue; }
        double acc[ORACLE_KMAX + 1][3];
        double accm[ORACLE_KMAX + 1], accn[ORACLE_KMAX + 1];
        for (int k = 0; k <= K; ++k) { acc[k][0] = acc[k][1] = acc[k][2] = 0.0; accm[k] = 0.0; accn[k] = 0.0; }
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r[ORACLE_KMAX + 1][3];
            for (int k = 0; k <= K; ++k)
                for (int c = 0; c < 3; ++c)
                    r[k][c] = path[((int64_t)k * 3 + c) * n + j] - path[((int64_t)k * 3 + c) * n + i];
            double w[ORACLE_KMAX + 2];
            w[0] = r[0][0] * r[0][0] + r[0][1] * r[0][1] + r[0][2] * r[0][2] + eps2;
            for (int m = 1; m <= K; ++m) {
                double s = 0.0;
                for (int l = 0; l <= m; ++l)
                    s += C[m][l] * (r[l][0] * r[m - l][0] + r[l][1] * r[m - l][1] + r[l][2] * r[m - l][2]);
                w[m] = s;
            }
            double u[ORACLE_KMAX + 1];
            u[0] = 1.0 / (w[0] * sqrt(w[0]));
            for (int m = 0; m < K; ++m) {
                double s1 = 0.0, s2 = 0.0;
                for (int k = 0; k <= m; ++k) s1 += C[m][k] * w[k + 1] * u[m - k];
                for (int k = 1; k <= m; ++k) s2 += C[m][k] * w[k] * u[m - k + 1];
                u[m + 1] = (-1.5 * s1 - s2) / w[0];
            }
            const double gm = G * mass[j];
            for (int m = 0; m <= K; ++m) {
                double t[3] = {0.0, 0.0, 0.0};
                for (int k = 0; k <= m; ++k)
                    for (int c = 0; c < 3; ++c) t[c] += C[m][k] * r[k][c] * u[m - k];
                for (int c = 0; c < 3; ++c) {
                    t[c] = gm * t[c];
                    acc[m][c] += t[c];
                }
                accm[m] += sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
            }
            if (nat) {
                /* natural derivative scale of this pair: G m_j s^-2 omega^k with
                   s = sqrt(r.r + eps^2), omega = max_k (|r^(k)| / s)^(1/k) */
                const double sft = sqrt(w[0]);
                double om = 0.0;
                for (int k = 1; k <= K; ++k) {
                    const double q = sqrt(r[k][0] * r[k][0] + r[k][1] * r[k][1] + r[k][2] * r[k][2]) / sft;
                    const double rate = pow(q, 1.0 / (double)k);
                    if (rate > om) om = rate;
                }
                double sc = fabs(gm) / w[0];
                for (int m = 0; m <= K; ++m) {
                    accn[m] += sc;
                    sc *= om;
                }
            }
        }
        for (int k = 0; k <= K; ++k) {
            for (int c = 0; c < 3; ++c) {
                out[((int64_t)k * 3 + c) * n_i + ii] = acc[k][c];
                if (!isfinite(acc[k][c])) bad |= 2;
            }
            if (mag) mag[(int64_t)k * n_i + ii] = accm[k];
            if (nat) nat[(int64_t)k * n_i + ii] = accn[k];
        }
    }
    if (bad & 1) return -1;
    if (bad & 2) return -2;
    return 0;
}

/*
 * phi[n_i]: phi_i = -sum_{j != i} G m_j / sqrt(|x_j - x_i|^2 + eps2)
 * x is [3][n].  Returns 0, -1 on bad arguments, -2 on a non-finite value.
 */
int oracle_potential(int64_t n, const double *mass, const double *x, double G, double eps2,
                     int64_t n_i, const int64_t *i_list, double *phi)
{
    if (n < 0 || eps2 < 0.0 || !mass || !x || !phi) return -1;
    if (!i_list) n_i = n;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(| : bad)
    for (int64_t ii = 0; ii < n_i; ++ii) {
        const int64_t i = i_list ? i_list[ii] : ii;
        if (i < 0 || i >= n) { bad |= 1; continue; }
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = x[j] - x[i], dy = x[n + j] - x[n + i], dz = x[2 * n + j] - x[2 * n + i];
            s -= G * mass[j] / sqrt(dx * dx + dy * dy + dz * dz + eps2);
        }
        phi[ii] = s;
        if (!isfinite(s)) bad |= 2;
    }
    if (bad & 1) return -1;
    if (bad & 2) return -2;
    return 0;
}

/* Number of OpenMP threads a parallel region uses (for reporting). */
int oracle_num_threads(void)
{
    int nt = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            nt = omp_get_num_threads();
#endif
        }
    }
    return nt;
}

/*
 * Largest pair "rate" of the time-step criterion (Sec. 3.3, Eq. 25):
 *   q = max_{i != j} G (m_i + m_j) / (r_ij^2 + eps^2)^(3/2),
 * so that H = eta * q^(-1/2) = eta * min_{i != j} ((r^2+eps^2)^(3/2) / (G (m_i+m_j)))^(1/2).
 * x is [3][n].  Returns 0 (with *qmax = 0 for n < 2), -1 on bad arguments.
 */
int oracle_max_pair_rate(int64_t n, const double *mass, const double *x, double G, double eps2, double *qmax)
{
    if (n < 0 || eps2 < 0.0 || !mass || !x || !qmax) return -1;
    double best = 0.0;
#pragma omp parallel for schedule(dynamic, 8) reduction(max : best)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = x[j] - x[i], dy = x[n + j] - x[n + i], dz = x[2 * n + j] - x[2 * n + i];
            const double w = dx * dx + dy * dy + dz * dz + eps2;
            const double q = G * (mass[i] + mass[j]) / (w * sqrt(w));
            if (q > best) best = q;
        }
    }
    *qmax = best;
    return 0;
}
