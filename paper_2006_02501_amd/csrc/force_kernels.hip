// O(N^2) evaluation of the softened pair acceleration and its time
// derivatives (the hot loop of every P(EC)^n iteration).
//
// Layout on the chip: a workgroup is 4 wave64 (256 lanes).  Each lane keeps
// IPT i-particles (their path x, v, a, adot and the running sums) in VGPRs;
// in the LDS-tiled kernel the four waves share the same 64*IPT i-particles
// and each takes a quarter of every j-tile, their sums being added through
// LDS at the end (4x fewer split partials than one i-set per lane).
// The workgroup walks its j-range in tiles of 256 j-particles; every tile is
// read from HBM once, coalesced (consecutive lanes, consecutive j), into LDS
// as one row per j (G m, then the path components), and every lane then
// reads the rows as wave-wide broadcasts.  The j-range is also split over
// gridDim.y workgroups so that a modest N still fills 256 CUs; those split
// partial sums are added in a fixed order by a second kernel (no atomics,
// bitwise reproducible).
//
// Chains: FP64 (everything double); Mixed (differences of the FP64 path in
// double, then cast; the r^-3 term and its derivative chain in float,
// summed in float over 32 j at a time and in double across those partial
// sums); Split (a and adot as in FP64, a^(2) and a^(3) as in Mixed, from the
// same FP64 differences); Generic (the FP64 recurrence up to the 5th
// derivative, for the initialisation).
#include "force_launch.h"
#include "pair_chain.h"

namespace hermite {
namespace {

template <int K>
struct Path {
    const double *p[K + 1];
};

constexpr int kFold = 32;   // mixed / split chains: j-particles per FP32 partial sum
constexpr int kWave = 64;   // lanes per wavefront

// Chains with FP32 partial sums (folded into FP64 every kFold j), and the
// first derivative order they keep in FP32.
template <Chain CH>
constexpr bool folds() { return CH == Chain::Mixed || CH == Chain::Split; }
template <Chain CH>
constexpr int first_f32() { return CH == Chain::Split ? 2 : 0; }

template <int K, Chain CH, int IPT>
__device__ __forceinline__ void fold_partials(double (&acc)[IPT][K + 1][3], float (&accf)[IPT][K + 1][3])
{
#pragma unroll
    for (int q = 0; q < IPT; ++q)
#pragma unroll
        for (int k = first_f32<CH>(); k <= K; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                acc[q][k][c] += (double)accf[q][k][c];
                accf[q][k][c] = 0.0f;
            }
}

// i-particles per workgroup of W waves: 64*IPT when the waves share them
// (and split the j-range), else 64*W*IPT.
constexpr int64_t iblock_size(int w, bool share, int ipt) { return (int64_t)(share ? kWave : kWave * w) * ipt; }

template <int K>
constexpr int row_stride() { return ((1 + 3 * (K + 1)) + 1) & ~1; }

// Running maximum, per i-particle, of the pair rate G (m_i + m_j) / (r^2 +
// eps^2)^(3/2) that sets the variable step of Sec. 3.3 (Eq. 25), taken along
// with the evaluation when QM (FP64 and split chains: one multiply, one FMA
// and one max per pair on the FP64 1/r they already have).
template <bool QM, int IPT>
struct RateMax {
    double gm[IPT];   // G m_i
    double q[IPT];
    __device__ __forceinline__ void add(int k, double mr3, double r3)
    {
        if constexpr (QM) q[k] = __builtin_fmax(q[k], __builtin_fma(gm[k], r3, mr3));
    }
};

// Largest rate over a workgroup of W waves (lanes past n give 0); thread 0
// writes it to qpart[blockIdx.y * gridDim.x + blockIdx.x].
template <bool QM, int IPT, int W>
__device__ __forceinline__ void store_rate(const RateMax<QM, IPT> &rm, const int64_t (&ii)[IPT], int64_t n,
                                           double *__restrict__ qpart)
{
    if constexpr (QM) {
        __shared__ double wq[W];
        double q = 0.0;
#pragma unroll
        for (int k = 0; k < IPT; ++k) q = ii[k] < n ? __builtin_fmax(q, rm.q[k]) : q;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) q = __builtin_fmax(q, __shfl_xor(q, off, 64));
        __syncthreads();
        if ((threadIdx.x & 63) == 0) wq[threadIdx.x >> 6] = q;
        __syncthreads();
        if (threadIdx.x == 0) {
            double r = wq[0];
#pragma unroll
            for (int w = 1; w < W; ++w) r = __builtin_fmax(r, wq[w]);
            qpart[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = r;
        }
    }
}

template <int K, Chain CH, int IPT, bool DIAG, bool QM, int UNROLL = 2>
__device__ __forceinline__ void tile_pass(const double *__restrict__ tile, const float *__restrict__ mtile, int cnt,
                                          int64_t j0, const int64_t (&ii)[IPT], const double (&xi)[IPT][K + 1][3],
                                          double eps2, double (&acc)[IPT][K + 1][3], float (&accf)[IPT][K + 1][3],
                                          RateMax<QM, IPT> &rm)
{
    constexpr int RS = row_stride<K>();
#pragma unroll UNROLL
    for (int jj = 0; jj < cnt; ++jj) {
        const double *row = tile + jj * RS;
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            const bool self = DIAG && (j0 + jj == ii[q]);
            if constexpr (CH == Chain::Fp64) {
                double r[3], v[3], a[3], j[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    r[c] = row[1 + c] - xi[q][0][c];
                    v[c] = row[4 + c] - xi[q][1][c];
                    if constexpr (K >= 2) a[c] = row[7 + c] - xi[q][2][c]; else a[c] = 0.0;
                    if constexpr (K >= 3) j[c] = row[10 + c] - xi[q][3][c]; else j[c] = 0.0;
                }
                double w = __builtin_fma(r[0], r[0], __builtin_fma(r[1], r[1], __builtin_fma(r[2], r[2], eps2)));
                double m = row[0];
                if (DIAG) {
                    w = self ? 1.0 : w;
                    m = self ? 0.0 : m;
                }
                const double rinv = rsqrt64(w);
                const double rinv2 = rinv * rinv;
                const double mr3 = m * rinv * rinv2;
                if constexpr (QM) rm.add(q, mr3, (DIAG && self) ? 0.0 : rinv * rinv2);
                chain_accumulate<K, double>(r, v, a, j, mr3, rinv2, acc[q]);
            } else if constexpr (CH == Chain::Mixed) {
                float r[3], v[3], a[3], j[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    r[c] = (float)(row[1 + c] - xi[q][0][c]);
                    v[c] = (float)(row[4 + c] - xi[q][1][c]);
                    if constexpr (K >= 2) a[c] = (float)(row[7 + c] - xi[q][2][c]); else a[c] = 0.0f;
                    if constexpr (K >= 3) j[c] = (float)(row[10 + c] - xi[q][3][c]); else j[c] = 0.0f;
                }
                float w = __builtin_fmaf(r[0], r[0], __builtin_fmaf(r[1], r[1], __builtin_fmaf(r[2], r[2], (float)eps2)));
                float m = mtile[jj];
                if (DIAG) {
                    w = self ? 1.0f : w;
                    m = self ? 0.0f : m;
                }
                const float rinv = rsqrt32(w);
                const float rinv2 = rinv * rinv;
                const float mr3 = m * rinv * rinv2;
                chain_accumulate<K, float>(r, v, a, j, mr3, rinv2, accf[q]);
            } else if constexpr (CH == Chain::Split) {
                double r[3], v[3];
                float a[3], j[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    r[c] = row[1 + c] - xi[q][0][c];
                    v[c] = row[4 + c] - xi[q][1][c];
                    a[c] = (float)(row[7 + c] - xi[q][2][c]);
                    if constexpr (K >= 3) j[c] = (float)(row[10 + c] - xi[q][3][c]); else j[c] = 0.0f;
                }
                double w = __builtin_fma(r[0], r[0], __builtin_fma(r[1], r[1], __builtin_fma(r[2], r[2], eps2)));
                double m = row[0];
                if (DIAG) {
                    w = self ? 1.0 : w;
                    m = self ? 0.0 : m;
                }
                const double rinv = rsqrt64(w);
                const double rinv2 = rinv * rinv;
                const double mr3 = m * rinv * rinv2;
                if constexpr (QM) rm.add(q, mr3, (DIAG && self) ? 0.0 : rinv * rinv2);
                chain_split<K>(r, v, a, j, mr3, rinv2, acc[q], accf[q]);
            } else {
                double r[K + 1][3];
#pragma unroll
                for (int k = 0; k <= K; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) r[k][c] = row[1 + 3 * k + c] - xi[q][k][c];
                generic_accumulate<K>(r, eps2, row[0], self, acc[q]);
            }
        }
    }
}

// Reduction of the W waves' partial sums through LDS, in wave order; wave 0
// ends up with the workgroup's sum.  buf holds (W-1)*IPT*(K+1)*3*64 doubles.
template <int K, int IPT, int W>
__device__ __forceinline__ void reduce_waves(double *buf, int wave, int lane, double (&acc)[IPT][K + 1][3])
{
    constexpr int NV = IPT * (K + 1) * 3;
    __syncthreads();
    if (wave > 0) {
        double *b = buf + (wave - 1) * NV * kWave;
#pragma unroll
        for (int q = 0; q < IPT; ++q)
#pragma unroll
            for (int k = 0; k <= K; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) b[((q * (K + 1) + k) * 3 + c) * kWave + lane] = acc[q][k][c];
    }
    __syncthreads();
    if (wave == 0) {
        for (int w = 0; w < W - 1; ++w)
#pragma unroll
            for (int q = 0; q < IPT; ++q)
#pragma unroll
                for (int k = 0; k <= K; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        acc[q][k][c] += buf[(w * NV + (q * (K + 1) + k) * 3 + c) * kWave + lane];
    }
}

// A workgroup is W wave64.  SHARE: the W waves share one block of 64*IPT
// i-particles and each takes its 64-row slice of every j-tile (their sums are
// added through LDS at the end); otherwise every lane has its own i-particles.
// A j-tile has 64*W rows, one loaded by each thread.
template <int K, Chain CH, int IPT, int W, bool SHARE, bool QM>
__global__ __launch_bounds__(kWave * W) void force_kernel(int64_t n, const double *__restrict__ mass, Path<K> path,
                                                          double G, double eps2, int64_t j_chunk, int k_first,
                                                          double *__restrict__ out, double *__restrict__ qpart,
                                                          int64_t i_base, int64_t i_lo, int64_t i_end)
{
    constexpr int RS = row_stride<K>();
    constexpr int UNR = 2;
    constexpr int TROWS = kWave * W;
    constexpr int TILE_D = TROWS * RS;
    constexpr int RED_D = SHARE ? (W - 1) * IPT * (K + 1) * 3 * kWave : 0;
    __shared__ __align__(16) double smem[TILE_D > RED_D ? TILE_D : RED_D];
    double *tile = smem;
    __shared__ float mtile[CH == Chain::Mixed ? TROWS : 1];
    const int tid = threadIdx.x;
    const int wave = tid / kWave, lane = tid % kWave;
    constexpr int ISTRIDE = SHARE ? kWave : kWave * W;
    constexpr int IBLK = ISTRIDE * IPT;
    // i-particles [i_lo, i_end) against every j.  The i-blocks stay on the
    // grid of the whole evaluation (i_base is a multiple of IBLK), so every
    // i takes exactly the operations it takes there; lanes outside the range
    // compute nothing that is stored.
    const int64_t ib0 = i_base + (int64_t)blockIdx.x * IBLK;
    const int64_t ib1 = min(n, ib0 + (int64_t)IBLK);
    const int64_t jbeg = (int64_t)blockIdx.y * j_chunk;
    const int64_t jend = min(n, jbeg + j_chunk);

    int64_t ii[IPT];
    double xi[IPT][K + 1][3];
    double acc[IPT][K + 1][3];
    float accf[IPT][K + 1][3];
    RateMax<QM, IPT> rm;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        ii[q] = ib0 + q * ISTRIDE + (SHARE ? lane : tid);
        const bool ok = ii[q] >= i_lo && ii[q] < i_end;
        if constexpr (QM) {
            rm.gm[q] = ok ? G * mass[ii[q]] : 0.0;
            rm.q[q] = 0.0;
        }
#pragma unroll
        for (int k = 0; k <= K; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                xi[q][k][c] = ok ? path.p[k][c * n + ii[q]] : 0.0;
                acc[q][k][c] = 0.0;
                accf[q][k][c] = 0.0f;
            }
    }

    for (int64_t j0 = jbeg; j0 < jend; j0 += TROWS) {
        const int cnt = (int)min((int64_t)TROWS, jend - j0);
        __syncthreads();
        if (tid < cnt) {
            const int64_t j = j0 + tid;
            double *row = tile + tid * RS;
            const double gm = G * mass[j];
            row[0] = gm;
            if constexpr (CH == Chain::Mixed) mtile[tid] = (float)gm;
#pragma unroll
            for (int k = 0; k <= K; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) row[1 + 3 * k + c] = path.p[k][c * n + j];
        }
        __syncthreads();
        const bool diag = (j0 < ib1) && (ib0 < j0 + cnt);
        // rows of this tile that this lane's wave handles
        const int r0 = SHARE ? min(cnt, wave * kWave) : 0;
        const int r1 = SHARE ? min(cnt, r0 + kWave) : cnt;
        if constexpr (!folds<CH>()) {
            if (r1 > r0) {
                if (diag)
                    tile_pass<K, CH, IPT, true, QM, UNR>(tile + r0 * RS, mtile, r1 - r0, j0 + r0, ii, xi, eps2, acc,
                                                         accf, rm);
                else
                    tile_pass<K, CH, IPT, false, QM, UNR>(tile + r0 * RS, mtile, r1 - r0, j0 + r0, ii, xi, eps2, acc,
                                                          accf, rm);
            }
        } else {
            // FP32 partial sums over kFold j at a time, folded into FP64: bounds
            // the rounding that small terms suffer next to a dominant one.
            for (int s0 = r0; s0 < r1; s0 += kFold) {
                const int cs = min(kFold, r1 - s0);
                if (diag)
                    tile_pass<K, CH, IPT, true, QM, UNR>(tile + s0 * RS, mtile + s0, cs, j0 + s0, ii, xi, eps2, acc,
                                                         accf, rm);
                else
                    tile_pass<K, CH, IPT, false, QM, UNR>(tile + s0 * RS, mtile + s0, cs, j0 + s0, ii, xi, eps2, acc,
                                                          accf, rm);
                fold_partials<K, CH, IPT>(acc, accf);
            }
        }
    }

    store_rate<QM, IPT, W>(rm, ii, i_end, qpart);
    if constexpr (SHARE) {
        reduce_waves<K, IPT, W>(smem, wave, lane, acc);
        if (wave != 0) return;
    }
    const int nv = K + 1 - k_first;
    double *o = out + (int64_t)blockIdx.y * nv * 3 * n;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (ii[q] < i_lo || ii[q] >= i_end) continue;
#pragma unroll
        for (int k = 0; k <= K; ++k) {
            if (k < k_first) continue;
#pragma unroll
            for (int c = 0; c < 3; ++c) o[((int64_t)(k - k_first) * 3 + c) * n + ii[q]] = acc[q][k][c];
        }
    }
}

// ---------------------------------------------------------------------------
// Scalar-stream variant.  Every lane of a wave needs the same j-particle at the
// same time, so the j-data is wave-uniform: it is packed once per evaluation
// into 128-byte records and read with scalar loads into SGPRs, which the VALU
// instructions take directly as operands.  No LDS, no barriers; the j-range
// is walked in three parts so only the part that overlaps the workgroup's own
// i-range pays for the self-term test.
constexpr int kJRec = kJRecDoubles;   // packed j-record: G m, x, v, a, adot, float G m, pad

template <int K>
__global__ __launch_bounds__(kBlock) void pack_j_kernel(int64_t n, const double *__restrict__ mass, Path<K> path,
                                                        double G, double *__restrict__ jrec)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    double rec[kJRec];
    const double gm = G * mass[j];
    rec[0] = gm;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) rec[1 + 3 * k + c] = k <= K ? path.p[k <= K ? k : 0][c * n + j] : 0.0;
    rec[13] = __builtin_bit_cast(double, (uint64_t)__builtin_bit_cast(uint32_t, (float)gm));
    rec[14] = 0.0;
    rec[15] = 0.0;
    double *dst = jrec + j * kJRec;
#pragma unroll
    for (int e = 0; e < kJRec; ++e) dst[e] = rec[e];
}

template <int K, Chain CH, int IPT, bool DIAG, bool QM>
__device__ __forceinline__ void stream_range(const double *__restrict__ jrec, int64_t jb, int64_t je,
                                             const int64_t (&ii)[IPT], const double (&xi)[IPT][K + 1][3],
                                             double eps2, double (&acc)[IPT][K + 1][3],
                                             float (&accf)[IPT][K + 1][3], RateMax<QM, IPT> &rm)
{
    if (jb >= je) return;
    constexpr int NJ = 1 + 3 * (K + 1);
    // Software pipeline: the scalar loads of record j+1 are issued before the
    // arithmetic of record j, so their latency hides behind it.
    double nx[NJ];
    uint64_t nxm;
#pragma unroll
    for (int e = 0; e < NJ; ++e) nx[e] = jrec[jb * kJRec + e];
    nxm = __builtin_bit_cast(uint64_t, jrec[jb * kJRec + 13]);
    for (int64_t j = jb; j < je; ++j) {
        double jd[NJ];
#pragma unroll
        for (int e = 0; e < NJ; ++e) jd[e] = nx[e];
        const float gmf = __builtin_bit_cast(float, (uint32_t)nxm);
        const int64_t jn = (j + 1 < je) ? j + 1 : j;
#pragma unroll
        for (int e = 0; e < NJ; ++e) nx[e] = jrec[jn * kJRec + e];
        nxm = __builtin_bit_cast(uint64_t, jrec[jn * kJRec + 13]);
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            const bool self = DIAG && (j == ii[q]);
            if constexpr (CH == Chain::Fp64) {
                double r[3], v[3], a[3], jk[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    r[c] = jd[1 + c] - xi[q][0][c];
                    v[c] = jd[4 + c] - xi[q][1][c];
                    if constexpr (K >= 2) a[c] = jd[7 + c] - xi[q][2][c]; else a[c] = 0.0;
                    if constexpr (K >= 3) jk[c] = jd[10 + c] - xi[q][3][c]; else jk[c] = 0.0;
                }
                double w = __builtin_fma(r[0], r[0], __builtin_fma(r[1], r[1], __builtin_fma(r[2], r[2], eps2)));
                double m = jd[0];
                if (DIAG) {
                    w = self ? 1.0 : w;
                    m = self ? 0.0 : m;
                }
                const double rinv = rsqrt64(w);
                const double rinv2 = rinv * rinv;
                if constexpr (QM) rm.add(q, m * rinv * rinv2, (DIAG && self) ? 0.0 : rinv * rinv2);
                chain_accumulate<K, double>(r, v, a, jk, m * rinv * rinv2, rinv2, acc[q]);
            } else if constexpr (CH == Chain::Split) {
                double r[3], v[3];
                float a[3], jk[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    r[c] = jd[1 + c] - xi[q][0][c];
                    v[c] = jd[4 + c] - xi[q][1][c];
                    a[c] = (float)(jd[7 + c] - xi[q][2][c]);
                    if constexpr (K >= 3) jk[c] = (float)(jd[10 + c] - xi[q][3][c]); else jk[c] = 0.0f;
                }
                double w = __builtin_fma(r[0], r[0], __builtin_fma(r[1], r[1], __builtin_fma(r[2], r[2], eps2)));
                double m = jd[0];
                if (DIAG) {
                    w = self ? 1.0 : w;
                    m = self ? 0.0 : m;
                }
                const double rinv = rsqrt64(w);
                const double rinv2 = rinv * rinv;
                if constexpr (QM) rm.add(q, m * rinv * rinv2, (DIAG && self) ? 0.0 : rinv * rinv2);
                chain_split<K>(r, v, a, jk, m * rinv * rinv2, rinv2, acc[q], accf[q]);
            } else {
                float r[3], v[3], a[3], jk[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    r[c] = (float)(jd[1 + c] - xi[q][0][c]);
                    v[c] = (float)(jd[4 + c] - xi[q][1][c]);
                    if constexpr (K >= 2) a[c] = (float)(jd[7 + c] - xi[q][2][c]); else a[c] = 0.0f;
                    if constexpr (K >= 3) jk[c] = (float)(jd[10 + c] - xi[q][3][c]); else jk[c] = 0.0f;
                }
                float w = __builtin_fmaf(r[0], r[0], __builtin_fmaf(r[1], r[1], __builtin_fmaf(r[2], r[2], (float)eps2)));
                float m = gmf;
                if (DIAG) {
                    w = self ? 1.0f : w;
                    m = self ? 0.0f : m;
                }
                const float rinv = rsqrt32(w);
                const float rinv2 = rinv * rinv;
                chain_accumulate<K, float>(r, v, a, jk, m * rinv * rinv2, rinv2, accf[q]);
            }
        }
    }
}

template <int K, Chain CH, int IPT, bool DIAG, bool QM>
__device__ __forceinline__ void stream_folded(const double *__restrict__ jrec, int64_t jb, int64_t je,
                                              const int64_t (&ii)[IPT], const double (&xi)[IPT][K + 1][3],
                                              double eps2, double (&acc)[IPT][K + 1][3],
                                              float (&accf)[IPT][K + 1][3], RateMax<QM, IPT> &rm)
{
    if constexpr (!folds<CH>()) {
        stream_range<K, CH, IPT, DIAG, QM>(jrec, jb, je, ii, xi, eps2, acc, accf, rm);
    } else {
        for (int64_t s0 = jb; s0 < je; s0 += kFold) {
            const int64_t s1 = min(je, s0 + (int64_t)kFold);
            stream_range<K, CH, IPT, DIAG, QM>(jrec, s0, s1, ii, xi, eps2, acc, accf, rm);
            fold_partials<K, CH, IPT>(acc, accf);
        }
    }
}

// W waves per workgroup.  SHARE: they share 64*IPT i-particles and each
// streams its own contiguous part of the workgroup's j-range (sums added
// through LDS); otherwise they stream the same records for different i.
template <int K, Chain CH, int IPT, int W, bool SHARE, bool QM>
__global__ __launch_bounds__(kWave * W) void force_stream_kernel(int64_t n, const double *__restrict__ jrec,
                                                                 Path<K> path, double eps2, int64_t j_chunk,
                                                                 double *__restrict__ out,
                                                                 const double *__restrict__ mass, double G,
                                                                 double *__restrict__ qpart, int64_t i_base,
                                                                 int64_t i_lo, int64_t i_end)
{
    __shared__ double red[SHARE ? (W - 1) * IPT * (K + 1) * 3 * kWave : 1];
    const int tid = threadIdx.x;
    const int wave = tid / kWave, lane = tid % kWave;
    constexpr int ISTRIDE = SHARE ? kWave : kWave * W;
    constexpr int IBLK = ISTRIDE * IPT;
    // i-particles [i_lo, i_end) against every j.  The i-blocks stay on the
    // grid of the whole evaluation (i_base is a multiple of IBLK), so every
    // i takes exactly the operations it takes there; lanes outside the range
    // compute nothing that is stored.
    const int64_t ib0 = i_base + (int64_t)blockIdx.x * IBLK;
    const int64_t ib1 = min(n, ib0 + (int64_t)IBLK);
    int64_t jbeg = (int64_t)blockIdx.y * j_chunk;
    int64_t jend = min(n, jbeg + j_chunk);
    if (SHARE) {
        // this wave's contiguous part of the workgroup's j-range
        const int64_t part = (max(jend - jbeg, (int64_t)0) + W - 1) / W;
        const int64_t wb = jbeg + wave * part;
        jend = min(jend, wb + part);
        jbeg = min(wb, jend);
    }

    int64_t ii[IPT];
    double xi[IPT][K + 1][3];
    double acc[IPT][K + 1][3];
    float accf[IPT][K + 1][3];
    RateMax<QM, IPT> rm;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        ii[q] = ib0 + q * ISTRIDE + (SHARE ? lane : tid);
        const bool ok = ii[q] >= i_lo && ii[q] < i_end;
        if constexpr (QM) {
            rm.gm[q] = ok ? G * mass[ii[q]] : 0.0;
            rm.q[q] = 0.0;
        }
#pragma unroll
        for (int k = 0; k <= K; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                xi[q][k][c] = ok ? path.p[k][c * n + ii[q]] : 0.0;
                acc[q][k][c] = 0.0;
                accf[q][k][c] = 0.0f;
            }
    }
    // [jbeg, d0) and [d1, jend) cannot contain one of this workgroup's i.
    const int64_t d0 = max(jbeg, min(jend, ib0));
    const int64_t d1 = max(d0, min(jend, ib1));
    stream_folded<K, CH, IPT, false, QM>(jrec, jbeg, d0, ii, xi, eps2, acc, accf, rm);
    stream_folded<K, CH, IPT, true, QM>(jrec, d0, d1, ii, xi, eps2, acc, accf, rm);
    stream_folded<K, CH, IPT, false, QM>(jrec, d1, jend, ii, xi, eps2, acc, accf, rm);

    store_rate<QM, IPT, W>(rm, ii, i_end, qpart);
    if constexpr (SHARE) {
        reduce_waves<K, IPT, W>(red, wave, lane, acc);
        if (wave != 0) return;
    }
    double *o = out + (int64_t)blockIdx.y * (K + 1) * 3 * n;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (ii[q] < i_lo || ii[q] >= i_end) continue;
#pragma unroll
        for (int k = 0; k <= K; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) o[((int64_t)k * 3 + c) * n + ii[q]] = acc[q][k][c];
    }
}

__global__ void reduce_splits_kernel(int64_t count, int nsplit, const double *__restrict__ partial,
                                     double *__restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    double s = partial[e];
#pragma unroll 8
    for (int sp = 1; sp < nsplit; ++sp) s += partial[(int64_t)sp * count + e];
    out[e] = s;
}

// The split partials of i-particles [i_off, i_off + ni) only (an evaluation of
// an i-range): element e = comp * ni + (i - i_off), comp over nc components.
__global__ void reduce_splits_range_kernel(int64_t n, int64_t i_off, int64_t ni, int nc, int nsplit,
                                           const double *__restrict__ partial, double *__restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nc * ni) return;
    const int64_t comp = e / ni;
    const int64_t idx = comp * n + i_off + (e - comp * ni);
    const int64_t count = (int64_t)nc * n;
    double s = partial[idx];
#pragma unroll 8
    for (int sp = 1; sp < nsplit; ++sp) s += partial[(int64_t)sp * count + idx];
    out[idx] = s;
}

// Workgroups of a launch (each writes one rate maximum when QM).
template <int IPT, int W, bool SHARE>
int64_t grid_blocks(int64_t n, int nsplit)
{
    const int64_t ib = iblock_size(W, SHARE, IPT);
    return (n + ib - 1) / ib * nsplit;
}

// i-particles of a launch: [i_off, i_off + i_count()) (all n by default)
int64_t i_count(const ForceArgs &a) { return a.i_cnt < 0 ? a.n : a.i_cnt; }

template <int IPT, int W, bool SHARE, bool QM>
bool rate_fits(const ForceArgs &a, int nsplit)
{
    if constexpr (!QM) return true;
    const int64_t nb = grid_blocks<IPT, W, SHARE>(i_count(a), nsplit);
    if (nb > a.qpart_cap) return false;
    if (a.q_count) *a.q_count = (int)nb;
    return true;
}

template <int K, Chain CH, int IPT, int W, bool SHARE, bool QM>
hipError_t launch_lds(const ForceArgs &a, int nsplit, int64_t j_chunk, double *dst, hipStream_t st)
{
    if (!rate_fits<IPT, W, SHARE, QM>(a, nsplit)) return hipErrorInvalidValue;
    Path<K> path;
    for (int k = 0; k <= K; ++k) path.p[k] = a.path[k];
    const int64_t ib = iblock_size(W, SHARE, IPT);
    const int64_t ni = i_count(a), base = a.i_off / ib * ib;
    dim3 grid((unsigned)((a.i_off + ni - base + ib - 1) / ib), (unsigned)nsplit);
    hipLaunchKernelGGL((force_kernel<K, CH, IPT, W, SHARE, QM>), grid, dim3(kWave * W), 0, st, a.n, a.mass, path,
                       a.G, a.eps2, j_chunk, a.k_first, dst, a.qpart, base, a.i_off, a.i_off + ni);
    return hipGetLastError();
}

template <int K, Chain CH, int IPT, int W, bool SHARE, bool QM>
hipError_t launch_stream(const ForceArgs &a, int nsplit, int64_t j_chunk, double *dst, hipStream_t st)
{
    if (!rate_fits<IPT, W, SHARE, QM>(a, nsplit)) return hipErrorInvalidValue;
    Path<K> path;
    for (int k = 0; k <= K; ++k) path.p[k] = a.path[k];
    hipLaunchKernelGGL((pack_j_kernel<K>), dim3((unsigned)((a.n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, a.n,
                       a.mass, path, a.G, a.jrec);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t ib = iblock_size(W, SHARE, IPT);
    const int64_t ni = i_count(a), base = a.i_off / ib * ib;
    dim3 grid((unsigned)((a.i_off + ni - base + ib - 1) / ib), (unsigned)nsplit);
    hipLaunchKernelGGL((force_stream_kernel<K, CH, IPT, W, SHARE, QM>), grid, dim3(kWave * W), 0, st, a.n,
                       (const double *)a.jrec, path, a.eps2, j_chunk, dst, a.mass, a.G, a.qpart, base, a.i_off,
                       a.i_off + ni);
    return hipGetLastError();
}

// Shapes: LDS source: 4 waves sharing an i-block; scalar source: 4 waves with
// their own i (sharing the streamed records) or 16 waves sharing an i-block
// (one i-particle per lane).
template <int K, Chain CH, bool QM>
hipError_t dispatch_k(const ForceArgs &a, const LaunchShape &sh, int nsplit, int64_t j_chunk, double *dst,
                      hipStream_t st)
{
    const bool scalar = sh.jsource == JSource::Scalar;
    if (sh.waves == 16) {
        // 1024-thread workgroups: 128 VGPRs per lane, which the LDS-tiled
        // kernel (its j-rows live in VGPRs) cannot meet without spilling.
        if (sh.ipt != 1 || !scalar) return hipErrorInvalidValue;
        return launch_stream<K, CH, 1, 16, true, QM>(a, nsplit, j_chunk, dst, st);
    }
    if (sh.waves != 4) return hipErrorInvalidValue;
    if (sh.ipt == 1)
        return scalar ? launch_stream<K, CH, 1, 4, false, QM>(a, nsplit, j_chunk, dst, st)
                      : launch_lds<K, CH, 1, 4, true, QM>(a, nsplit, j_chunk, dst, st);
    if (sh.ipt == 2)
        return scalar ? launch_stream<K, CH, 2, 4, false, QM>(a, nsplit, j_chunk, dst, st)
                      : launch_lds<K, CH, 2, 4, true, QM>(a, nsplit, j_chunk, dst, st);
    // 3 or 4 i-particles per lane: scalar source only (the LDS kernel's
    // j-rows would not fit beside them in VGPRs)
    if (!scalar) return hipErrorInvalidValue;
    if (sh.ipt == 3) return launch_stream<K, CH, 3, 4, false, QM>(a, nsplit, j_chunk, dst, st);
    if (sh.ipt == 4) return launch_stream<K, CH, 4, 4, false, QM>(a, nsplit, j_chunk, dst, st);
    return hipErrorInvalidValue;
}

template <Chain CH, bool QM>
hipError_t dispatch(const ForceArgs &a, const LaunchShape &sh, int nsplit, int64_t j_chunk, double *dst,
                    hipStream_t st)
{
    if constexpr (CH == Chain::Generic) {
        switch (a.K) {
            case 1: return launch_lds<1, CH, 1, 4, false, false>(a, nsplit, j_chunk, dst, st);
            case 3: return launch_lds<3, CH, 1, 4, false, false>(a, nsplit, j_chunk, dst, st);
            case 5: return launch_lds<5, CH, 1, 4, false, false>(a, nsplit, j_chunk, dst, st);
            default: return hipErrorInvalidValue;
        }
    } else if constexpr (CH == Chain::Split) {
        // 4th order has no FP32 part: the split chain is the FP64 one
        switch (a.K) {
            case 1: return dispatch_k<1, Chain::Fp64, QM>(a, sh, nsplit, j_chunk, dst, st);
            case 2: return dispatch_k<2, CH, QM>(a, sh, nsplit, j_chunk, dst, st);
            case 3: return dispatch_k<3, CH, QM>(a, sh, nsplit, j_chunk, dst, st);
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (a.K) {
            case 1: return dispatch_k<1, CH, QM>(a, sh, nsplit, j_chunk, dst, st);
            case 2: return dispatch_k<2, CH, QM>(a, sh, nsplit, j_chunk, dst, st);
            case 3: return dispatch_k<3, CH, QM>(a, sh, nsplit, j_chunk, dst, st);
            default: return hipErrorInvalidValue;
        }
    }
}

}  // namespace

int64_t shape_iblock(const LaunchShape &sh, bool generic)
{
    if (generic) return iblock_size(4, false, 1);
    const bool share = sh.waves == 16 || sh.jsource == JSource::Lds;
    return iblock_size(sh.waves, share, sh.ipt);
}

int auto_split(int64_t n, const LaunchShape &sh, bool generic)
{
    if (n <= 0) return 1;
    const int64_t ib = shape_iblock(sh, generic);
    const int64_t iblocks = (n + ib - 1) / ib;
    // aim at 4096 resident waves (16 per CU) in one pass
    const int64_t waves_per_wg = generic ? 4 : sh.waves;
    const int64_t target = 4096 / waves_per_wg;
    int64_t s = (target + iblocks - 1) / iblocks;
    const int64_t tiles = (n + kTile - 1) / kTile;
    if (s > tiles) s = tiles;
    if (s > 64) s = 64;
    if (s < 1) s = 1;
    return (int)s;
}

hipError_t launch_force(const ForceArgs &a, Chain chain, const LaunchShape &sh, int nsplit, hipStream_t st)
{
    if (a.n <= 0) return hipSuccess;
    const int nv = a.K + 1 - a.k_first;
    if (nv <= 0 || a.K >= kMaxPath) return hipErrorInvalidValue;
    const bool generic = chain == Chain::Generic;
    if (!generic && (a.k_first != 0 || a.K > 3)) return hipErrorInvalidValue;
    const bool ranged = a.i_off != 0 || a.i_cnt >= 0;
    if (ranged && (a.i_off < 0 || a.i_cnt < 0 || a.i_off + a.i_cnt > a.n || a.qpart)) return hipErrorInvalidValue;
    if (ranged && a.i_cnt == 0) return hipSuccess;
    if (sh.jsource == JSource::Pairs) {
        // every pair once covers all bodies; an i-range takes the one-sided kernels
        if (generic || sh.ipt != 1 || sh.waves != 4 || ranged) return hipErrorInvalidValue;
        return launch_force_pairs(a, chain, st);
    }
    if (!generic && sh.jsource == JSource::Scalar && !a.jrec) return hipErrorInvalidValue;
    const int64_t per_split = (int64_t)nv * 3 * a.n;
    if (nsplit < 1) nsplit = 1;
    if (nsplit > 1 && (int64_t)nsplit * per_split > a.partial_cap) {
        nsplit = (int)(a.partial_cap / per_split);
        if (nsplit < 2) nsplit = 1;
    }
    int64_t j_chunk = (a.n + nsplit - 1) / nsplit;
    j_chunk = (j_chunk + kTile - 1) / kTile * kTile;
    nsplit = (int)((a.n + j_chunk - 1) / j_chunk);
    double *dst = nsplit > 1 ? a.partial : a.out;
    hipError_t e;
    // the fused pair-rate maximum: FP64 and split chains only
    const bool qm = a.qpart != nullptr;
    if (qm && chain != Chain::Fp64 && chain != Chain::Split) return hipErrorInvalidValue;
    switch (chain) {
        case Chain::Fp64:
            e = qm ? dispatch<Chain::Fp64, true>(a, sh, nsplit, j_chunk, dst, st)
                   : dispatch<Chain::Fp64, false>(a, sh, nsplit, j_chunk, dst, st);
            break;
        case Chain::Mixed: e = dispatch<Chain::Mixed, false>(a, sh, nsplit, j_chunk, dst, st); break;
        case Chain::Split:
            e = qm ? dispatch<Chain::Split, true>(a, sh, nsplit, j_chunk, dst, st)
                   : dispatch<Chain::Split, false>(a, sh, nsplit, j_chunk, dst, st);
            break;
        default: e = dispatch<Chain::Generic, false>(a, sh, nsplit, j_chunk, dst, st); break;
    }
    if (e != hipSuccess || nsplit == 1) return e;
    if (ranged) {
        const int64_t cnt = (int64_t)nv * 3 * a.i_cnt;
        hipLaunchKernelGGL(reduce_splits_range_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, a.n,
                           a.i_off, a.i_cnt, nv * 3, nsplit, (const double *)a.partial, a.out);
        return hipGetLastError();
    }
    const int64_t blocks = (per_split + 255) / 256;
    hipLaunchKernelGGL(reduce_splits_kernel, dim3((unsigned)blocks), dim3(256), 0, st, per_split, nsplit,
                       (const double *)a.partial, a.out);
    return hipGetLastError();
}

}  // namespace hermite
