// O(N^2) evaluation with every pair taken once: the pair's chain serves
// both bodies (Newton's third law extended to the derivatives: the vectors
// r, J', S', C' change sign under i <-> j, the scalars alpha, beta, gamma do
// not), so the chain runs N (N - 1) / 2 times instead of N (N - 1).  Chains:
// FP64; mixed (FP64 differences, then the FP32 chain); split (orders 0 and 1
// as in FP64, bitwise, orders 2 and 3 in FP32).
//
// Work items are pairs (I, J), I <= J, of super-blocks of 256 bodies; one
// workgroup of 4 wave64 per item.  Wave w keeps the 64 bodies of i-block w of
// super-block I (path and running sums) in VGPRs.  The j super-block is staged
// in LDS (structure of arrays, G m then the path components).  In phase s,
// wave w sweeps j-block v = (w + s) mod 4: at sweep step t lane l pairs its
// body with j-body (l + t) mod 64, and the j-body's running sum travels with
// it: after every step the j-sums move one lane down (DPP wave rotate), so the
// lane that handles a j-body next step holds its sum.  After the sweep the
// wave adds its j-sums into the LDS sums of block v, which no other wave
// touches in that phase (the phases form a Latin square); a barrier separates
// the phases.  On the diagonal item (I = J) each unordered pair of blocks is
// visited once (phases 0, 1, and 2 for waves 0 and 1 only), and inside a
// block each unordered pair of bodies once (steps 1..32, step 32 on lanes
// 0..31 only).  FP32 sums (mixed, and split orders 2 and 3) cover at most 32
// steps: then the i-side folds into its FP64 sums and the j-side into the LDS
// sums (the same 32-term bound as the other kernels' FP32 partial sums).
//
// Outputs per item: the i-side sums of super-block I and the j-side sums of
// super-block J (partial sums in HBM); a second kernel adds, for every body,
// the partials of the items that hold it, in a fixed order.  No atomics:
// the result is bitwise reproducible.  A launch of few items (at most half
// as many as the GPU holds at once, up to ~6900 bodies) takes one workgroup
// per item and phase instead, each writing its own partials: four times the
// workgroups for a GPU that would otherwise run latency-bound.  With two or
// more waves per SIMD a SIMD issues nearly as fast as with three, so larger
// launches, partial last round included, gain nothing from it (measured at
// 8k-32k bodies).  The partials take 2 * 12 * 256 doubles
// per item, about N^2 / 2700 doubles in all (100 MB at N = 16384), so one
// launch covers at most kPairsMaxN bodies; beyond that the bodies are cut into
// chunks and every pair of chunks is one launch (a triangle or a rectangle of
// items) whose partials are added to the output in a fixed order.
#include <algorithm>
#include <atomic>
#include <type_traits>

#include "force_launch.h"
#include "lane_moves.h"
#include "pair_chain.h"

namespace hermite {
namespace {

constexpr int kPW = 4;             // waves per workgroup = j-blocks per super-block
constexpr int kPL = 64;            // lanes per wave = bodies per block
constexpr int kPS = kPW * kPL;     // bodies per super-block
constexpr int kMaxDevices = 64;    // devices whose resident-workgroup counts are cached

template <int K>
struct PPath {
    const double *p[K + 1];
};

// First derivative order a chain sums in FP32 (K + 1: none).
template <Chain CH, int K>
constexpr int f32_from() { return CH == Chain::Mixed ? 0 : CH == Chain::Split ? 2 : K + 1; }

// Item k -> (I, J): the NS (NS - 1) / 2 off-diagonal items first, row by
// row, then the NS diagonal ones (they carry ~5/8 of an item's work and end
// the launch).
__device__ __forceinline__ void item_pair(int64_t k, int ns, int &I, int &J)
{
    const int64_t offd = (int64_t)ns * (ns - 1) / 2;
    if (k >= offd) {
        I = J = (int)(k - offd);
        return;
    }
    int i = 0;
    int64_t off = 0;
    while (off + (ns - 1 - i) <= k) {
        off += ns - 1 - i;
        ++i;
    }
    I = i;
    J = i + 1 + (int)(k - off);
}

__device__ __forceinline__ int64_t item_index(int I, int J, int ns)
{
    if (I == J) return (int64_t)ns * (ns - 1) / 2 + I;
    return (int64_t)I * (ns - 1) - (int64_t)I * (I - 1) / 2 + (J - I - 1);
}

// The super-block pairs of one launch: the triangle I <= J of one chunk of
// nsi super-blocks starting at ci0 (tri), or the whole rectangle of chunk
// ci0 (nsi super-blocks) against chunk cj0 (nsj super-blocks).
struct PairsGrid {
    int ci0, nsi, cj0, nsj;
    int tri;
};

// Three workgroups per CU fit the LDS; the register cap that lets them all be
// resident costs the 8th-order FP64 kernel a few spilled bytes and is still
// faster (609 against 637 us on the 16k disc) than two per CU.
// SPLIT: workgroup b takes phase b % 4 of item b / 4 (and writes partials of
// its own); otherwise workgroup b takes item b whole.
template <int K, Chain CH, bool QM, bool SPLIT>
__global__ __launch_bounds__(kPS, 3) void force_pairs_kernel(int64_t n, const double *__restrict__ mass, PPath<K> path,
                                                          double G, double eps2, PairsGrid pg,
                                                          double *__restrict__ part, double *__restrict__ qpart)
{
    constexpr int NV = (K + 1) * 3;
    constexpr int F = f32_from<CH, K>();   // orders F..K are summed in FP32 first
    constexpr int kFoldSteps = 32;         // sweep steps per FP32 partial sum
    __shared__ double sj[NV + 1][kPS];     // j super-block: G m, then x, v, (a, adot) components
    __shared__ double jsum[NV][kPS];       // j-side sums of the item
    __shared__ float sjm[CH == Chain::Mixed ? kPS : 1];   // FP32 G m (mixed chain)
    __shared__ double wq[kPW];
    const int tid = threadIdx.x;
    const int w = tid / kPL, l = tid % kPL;
    const int64_t item = SPLIT ? (int64_t)blockIdx.x / kPW : (int64_t)blockIdx.x;
    int I, J;   // super-blocks, relative to their chunks
    if (pg.tri) {
        item_pair(item, pg.nsi, I, J);
    } else {
        I = (int)(item / pg.nsj);
        J = (int)(item % pg.nsj);
    }
    const bool diag = pg.tri && I == J;
    I += pg.ci0;
    J += pg.cj0;

    const int64_t jg = (int64_t)J * kPS + tid;
    const bool jok = jg < n;
    const double gmj_own = jok ? G * mass[jg] : 0.0;
    sj[0][tid] = gmj_own;
    if constexpr (CH == Chain::Mixed) sjm[tid] = (float)gmj_own;
#pragma unroll
    for (int k = 0; k <= K; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) sj[1 + 3 * k + c][tid] = jok ? path.p[k][c * n + jg] : 0.0;
#pragma unroll
    for (int e = 0; e < NV; ++e) jsum[e][tid] = 0.0;

    const int64_t ig = (int64_t)I * kPS + tid;
    const bool iok = ig < n;
    const double gmi = iok ? G * mass[ig] : 0.0;
    const float gmif = (float)gmi;
    double xi[K + 1][3], acc_i[K + 1][3];
    float accf_i[K + 1][3];
#pragma unroll
    for (int k = 0; k <= K; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xi[k][c] = iok ? path.p[k][c * n + ig] : 0.0;
            acc_i[k][c] = 0.0;
            accf_i[k][c] = 0.0f;
        }
    double qmax = 0.0;
    // j-bodies of super-block J that exist; an item with padding bodies on
    // either side (the last super-block of a ragged n) masks their lanes
    const int jvalid = (int)min((int64_t)kPS, n - (int64_t)J * kPS);
    const bool edge = jvalid < kPS || (int64_t)(I + 1) * kPS > n;
    __syncthreads();

    const int nphase = diag ? 3 : kPW;
    const int s_lo = SPLIT ? (int)(blockIdx.x % kPW) : 0;
    const int s_hi = SPLIT ? min(s_lo + 1, nphase) : nphase;
    for (int s = s_lo; s < s_hi; ++s) {
        const int v = (w + s) % kPW;
        const bool same = diag && s == 0;                 // the wave's own block
        if (!(diag && s == 2 && w >= 2)) {                // wave-uniform
            double acc_j[K + 1][3];
            float accf_j[K + 1][3];
#pragma unroll
            for (int k = 0; k <= K; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    acc_j[k][c] = 0.0;
                    accf_j[k][c] = 0.0f;
                }
            const int t0 = same ? 1 : 0, t1 = same ? kPL / 2 : kPL - 1;
            // one sweep step; MASKED: some lanes may have to drop their pair
            auto step = [&](int t, auto masked) {
                const int js = v * kPL + ((l + t) & (kPL - 1));
                // (unmasked steps: every lane's pair counts)
                const bool ok = !decltype(masked)::value ||
                                (iok && js < jvalid && !(same && t == kPL / 2 && l >= kPL / 2));
                // relative path (FP64 differences)
                double d[K + 1][3];
#pragma unroll
                for (int k = 0; k <= K; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) d[k][c] = sj[1 + 3 * k + c][js] - xi[k][c];
                if constexpr (decltype(masked)::value) {
                    // a lane that must not count its pair (a padding body, or
                    // the second half of step 32) takes a zero path, so its
                    // chain is exactly zero: evaluated at w = 1 on the real
                    // differences it could overflow FP32 and give 0 * inf
#pragma unroll
                    for (int k = 0; k <= K; ++k)
#pragma unroll
                        for (int c = 0; c < 3; ++c) d[k][c] = ok ? d[k][c] : 0.0;
                }
                if constexpr (CH == Chain::Mixed) {
                    float r[3], vv[3], a[3], jk[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        r[c] = (float)d[0][c];
                        vv[c] = (float)d[1][c];
                        if constexpr (K >= 2) a[c] = (float)d[K >= 2 ? 2 : 0][c]; else a[c] = 0.0f;
                        if constexpr (K >= 3) jk[c] = (float)d[K >= 3 ? 3 : 0][c]; else jk[c] = 0.0f;
                    }
                    float w2 = __builtin_fmaf(r[0], r[0],
                                              __builtin_fmaf(r[1], r[1], __builtin_fmaf(r[2], r[2], (float)eps2)));
                    w2 = ok ? w2 : 1.0f;
                    const float rinv = rsqrt32(w2);
                    const float rinv2 = rinv * rinv;
                    const float q3 = ok ? rinv * rinv2 : 0.0f;
                    if constexpr (QM) {
                        // the step criterion's rate, from the FP64 differences
                        double w64 = __builtin_fma(d[0][0], d[0][0],
                                                   __builtin_fma(d[0][1], d[0][1], __builtin_fma(d[0][2], d[0][2], eps2)));
                        w64 = ok ? w64 : 1.0;
                        const double y = rsqrt64(w64);
                        qmax = __builtin_fmax(qmax, ok ? (gmi + sj[0][js]) * (y * y * y) : 0.0);
                    }
                    chain_pair<K, float>(r, vv, a, jk, sjm[js] * q3, -gmif * q3, rinv2, accf_i, accf_j);
                } else {
                    double r[3], vv[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        r[c] = d[0][c];
                        vv[c] = d[1][c];
                    }
                    double w2 =
                        __builtin_fma(r[0], r[0], __builtin_fma(r[1], r[1], __builtin_fma(r[2], r[2], eps2)));
                    w2 = ok ? w2 : 1.0;
                    const double rinv = rsqrt64(w2);
                    const double rinv2 = rinv * rinv;
                    const double q3 = ok ? rinv * rinv2 : 0.0;
                    const double gmj = sj[0][js];
                    if constexpr (QM) qmax = __builtin_fmax(qmax, (gmi + gmj) * q3);
                    if constexpr (CH == Chain::Split) {
                        float a[3], jk[3];
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            a[c] = (float)d[K >= 2 ? 2 : 0][c];
                            if constexpr (K >= 3) jk[c] = (float)d[K >= 3 ? 3 : 0][c]; else jk[c] = 0.0f;
                        }
                        chain_split_pair<K>(r, vv, a, jk, gmj * q3, -gmi * q3, rinv2, acc_i, acc_j, accf_i,
                                            accf_j);
                    } else {
                        double a[3], jk[3];
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            if constexpr (K >= 2) a[c] = d[K >= 2 ? 2 : 0][c]; else a[c] = 0.0;
                            if constexpr (K >= 3) jk[c] = d[K >= 3 ? 3 : 0][c]; else jk[c] = 0.0;
                        }
                        chain_pair<K, double>(r, vv, a, jk, gmj * q3, -gmi * q3, rinv2, acc_i, acc_j);
                    }
                }
#pragma unroll
                for (int k = 0; k <= K; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        if (k < F) acc_j[k][c] = lane_down(acc_j[k][c]);
                        else accf_j[k][c] = lane_down(accf_j[k][c]);
                    }
                            };
            for (int tc = t0; tc <= t1; tc += kFoldSteps) {
                const int te = min(t1, tc + kFoldSteps - 1);
                if (edge) {
                    for (int t = tc; t <= te; ++t) step(t, std::true_type{});
                } else {
                    // the diagonal sweep's last step (32) counts its pairs on
                    // lanes 0..31 only
                    const int tn = (same && te == kPL / 2) ? te - 1 : te;
                    for (int t = tc; t <= tn; ++t) step(t, std::false_type{});
                    if (tn < te) step(te, std::true_type{});
                }
                if constexpr (F <= K) {
                    // fold the FP32 sums of these steps: the i-side into its FP64
                    // sums, the j-side (now held by the lane of j-body
                    // (l + te + 1) mod 64) into the LDS sums of block v
                    const int jf = v * kPL + ((l + te + 1) & (kPL - 1));
#pragma unroll
                    for (int k = F; k <= K; ++k)
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            acc_i[k][c] += (double)accf_i[k][c];
                            accf_i[k][c] = 0.0f;
                            jsum[3 * k + c][jf] += (double)accf_j[k][c];
                            accf_j[k][c] = 0.0f;
                        }
                }
            }
            if constexpr (F > 0) {
                // lane l now holds the FP64 sums of j-body (l + t1 + 1) mod 64 of block v
                const int js_end = v * kPL + ((l + t1 + 1) & (kPL - 1));
#pragma unroll
                for (int k = 0; k < F && k <= K; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) jsum[3 * k + c][js_end] += acc_j[k][c];
            }
        }
        __syncthreads();
    }

    // partials of this workgroup: [2][NV][kPS], side 0 = super-block I, 1 = J
    double *pi = part + (int64_t)blockIdx.x * 2 * NV * kPS;
#pragma unroll
    for (int k = 0; k <= K; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            pi[(3 * k + c) * kPS + tid] = acc_i[k][c];
            pi[(NV + 3 * k + c) * kPS + tid] = jsum[3 * k + c][tid];
        }
    if constexpr (QM) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) qmax = __builtin_fmax(qmax, __shfl_xor(qmax, off, 64));
        if (l == 0) wq[w] = qmax;
        __syncthreads();
        if (tid == 0) {
            double q = wq[0];
#pragma unroll
            for (int k = 1; k < kPW; ++k) q = __builtin_fmax(q, wq[k]);
            qpart[blockIdx.x] = q;
        }
    }
}

// Partial of item k at p (one side and component): its workgroup's, or with
// SPLIT the sum of its four phase workgroups' in phase order.
template <bool SPLIT>
__device__ __forceinline__ double item_part(const double *__restrict__ p, int64_t k, int64_t stride)
{
    if constexpr (!SPLIT) {
        return p[k * stride];
    } else {
        double t = p[kPW * k * stride];
#pragma unroll
        for (int ph = 1; ph < kPW; ++ph) t += p[(kPW * k + ph) * stride];
        return t;
    }
}

// Every body's sums (one launch covering all of them, the triangle of the
// single chunk): the i-side partials of the items (Kb, J), J = Kb..NS-1, then
// the j-side partials of the items (I, Kb), I = 0..Kb, in that order.
template <bool SPLIT>
__global__ void reduce_pairs_kernel(int64_t n, int nv, int ns, const double *__restrict__ part,
                                    double *__restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nv * n) return;
    const int comp = (int)(e / n);
    const int64_t b = e - (int64_t)comp * n;
    const int kb = (int)(b / kPS), loc = (int)(b % kPS);
    const int64_t stride = (int64_t)2 * nv * kPS;
    // (unrolled so that several loads are in flight; the additions keep their order)
    double s = 0.0;
#pragma unroll 8
    for (int J = kb; J < ns; ++J) s += item_part<SPLIT>(part + (int64_t)comp * kPS + loc, item_index(kb, J, ns), stride);
#pragma unroll 8
    for (int I = 0; I <= kb; ++I)
        s += item_part<SPLIT>(part + (int64_t)(nv + comp) * kPS + loc, item_index(I, kb, ns), stride);
    out[e] = s;
}

// One launch of a chunked evaluation: adds, for every body of its chunk(s),
// the partials of that launch's items that hold it (the same order as above
// within a triangle; J ascending for the i-side and I ascending for the
// j-side of a rectangle) to out.
__global__ void reduce_pairs_add_kernel(int64_t n, int nv, PairsGrid pg, const double *__restrict__ part,
                                        double *__restrict__ out)
{
    const int64_t nba = min((int64_t)pg.nsi * kPS, n - (int64_t)pg.ci0 * kPS);
    const int64_t nbb = pg.tri ? 0 : min((int64_t)pg.nsj * kPS, n - (int64_t)pg.cj0 * kPS);
    const int64_t nb = nba + nbb;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nv * nb) return;
    const int comp = (int)(e / nb);
    const int64_t r = e - (int64_t)comp * nb;
    const int64_t stride = (int64_t)2 * nv * kPS;
    double s = 0.0;
    int64_t body;
    if (r < nba) {
        const int kb = (int)(r / kPS), loc = (int)(r % kPS);
        body = (int64_t)pg.ci0 * kPS + r;
        if (pg.tri) {
#pragma unroll 8
            for (int J = kb; J < pg.nsi; ++J)
                s += part[item_index(kb, J, pg.nsi) * stride + (int64_t)comp * kPS + loc];
#pragma unroll 8
            for (int I = 0; I <= kb; ++I)
                s += part[item_index(I, kb, pg.nsi) * stride + (int64_t)(nv + comp) * kPS + loc];
        } else {
#pragma unroll 8
            for (int J = 0; J < pg.nsj; ++J)
                s += part[((int64_t)kb * pg.nsj + J) * stride + (int64_t)comp * kPS + loc];
        }
    } else {
        const int64_t rb = r - nba;
        const int kb = (int)(rb / kPS), loc = (int)(rb % kPS);
        body = (int64_t)pg.cj0 * kPS + rb;
#pragma unroll 8
        for (int I = 0; I < pg.nsi; ++I)
            s += part[((int64_t)I * pg.nsj + kb) * stride + (int64_t)(nv + comp) * kPS + loc];
    }
    out[(int64_t)comp * n + body] += s;
}

__global__ void zero_kernel(int64_t count, double *__restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) out[e] = 0.0;
}

// Workgroups of this kernel the current device holds at once (0 if the
// query fails: then nothing is split); cached per device.
template <int K, Chain CH, bool QM>
int64_t resident_slots()
{
    static std::atomic<int> cache[kMaxDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 0;
    int v = cache[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, force_pairs_kernel<K, CH, QM, true>, kPS, 0) !=
                hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        v = std::max(per_cu * cus, 0);
        cache[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

template <int K, Chain CH, bool QM>
hipError_t launch_k(const ForceArgs &a, hipStream_t st)
{
    PPath<K> path;
    for (int k = 0; k <= K; ++k) path.p[k] = a.path[k];
    const int ns = (int)((a.n + kPS - 1) / kPS);
    const int nv = (K + 1) * 3;
    if (a.n <= kPairsMaxN && pairs_items(a.n) * 2 * nv * kPS <= a.partial_cap) {
        // one launch: the triangle of all super-blocks, one workgroup per
        // item and phase when the items are few and the workspace holds it
        const PairsGrid pg{0, ns, 0, ns, 1};
        const int64_t items = pairs_items(a.n);
        const bool split = pairs_split(items, resident_slots<K, CH, QM>()) &&
                           kPW * items * 2 * nv * kPS <= a.partial_cap && (!QM || kPW * items <= a.qpart_cap);
        const int64_t wgs = split ? kPW * items : items;
        if (QM && a.q_count) *a.q_count = (int)wgs;
        if (split)
            hipLaunchKernelGGL((force_pairs_kernel<K, CH, QM, true>), dim3((unsigned)wgs), dim3(kPS), 0, st, a.n,
                               a.mass, path, a.G, a.eps2, pg, a.partial, a.qpart);
        else
            hipLaunchKernelGGL((force_pairs_kernel<K, CH, QM, false>), dim3((unsigned)wgs), dim3(kPS), 0, st, a.n,
                               a.mass, path, a.G, a.eps2, pg, a.partial, a.qpart);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int64_t cnt = (int64_t)nv * a.n;
        const dim3 rg((unsigned)((cnt + 255) / 256));
        if (split)
            hipLaunchKernelGGL(reduce_pairs_kernel<true>, rg, dim3(256), 0, st, a.n, nv, ns,
                               (const double *)a.partial, a.out);
        else
            hipLaunchKernelGGL(reduce_pairs_kernel<false>, rg, dim3(256), 0, st, a.n, nv, ns,
                               (const double *)a.partial, a.out);
        return hipGetLastError();
    }
    // chunks of cs super-blocks, as large as the workspace holds a rectangle
    // of (up to 64 x 64 items); chunk pairs in a fixed order, each adding its
    // partials into the zeroed output
    const int cs = pairs_chunk(a.partial_cap, K);
    const int nc = (ns + cs - 1) / cs;
    const int64_t cnt = (int64_t)nv * a.n;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, cnt, a.out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int A = 0; A < nc; ++A)
        for (int B = A; B < nc; ++B) {
            PairsGrid pg{A * cs, min(cs, ns - A * cs), B * cs, min(cs, ns - B * cs), A == B ? 1 : 0};
            const int64_t items = pg.tri ? (int64_t)pg.nsi * (pg.nsi + 1) / 2 : (int64_t)pg.nsi * pg.nsj;
            hipLaunchKernelGGL((force_pairs_kernel<K, CH, false, false>), dim3((unsigned)items), dim3(kPS), 0, st, a.n,
                               a.mass, path, a.G, a.eps2, pg, a.partial, (double *)nullptr);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
            const int64_t nb = (int64_t)pg.nsi * kPS + (pg.tri ? 0 : (int64_t)pg.nsj * kPS);
            const int64_t rc = (int64_t)nv * nb;
            hipLaunchKernelGGL(reduce_pairs_add_kernel, dim3((unsigned)((rc + 255) / 256)), dim3(256), 0, st, a.n,
                               nv, pg, (const double *)a.partial, a.out);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

template <Chain CH, bool QM>
hipError_t launch_chain(const ForceArgs &a, hipStream_t st)
{
    switch (a.K) {
        case 1: return launch_k<1, CH == Chain::Split ? Chain::Fp64 : CH, QM>(a, st);   // split = FP64 at 4th order
        case 2: return launch_k<2, CH, QM>(a, st);
        default: return launch_k<3, CH, QM>(a, st);
    }
}

}  // namespace

int64_t pairs_items(int64_t n)
{
    const int64_t ns = (n + kPS - 1) / kPS;
    return ns * (ns + 1) / 2;
}

bool pairs_split(int64_t items, int64_t slots) { return slots > 0 && 2 * items <= slots; }

namespace {
template <int K>
int64_t max_slots()
{
    constexpr Chain kSplit = K == 1 ? Chain::Fp64 : Chain::Split;
    return std::max({resident_slots<K, Chain::Fp64, false>(), resident_slots<K, Chain::Fp64, true>(),
                     resident_slots<K, Chain::Mixed, false>(), resident_slots<K, Chain::Mixed, true>(),
                     resident_slots<K, kSplit, false>(), resident_slots<K, kSplit, true>()});
}
}  // namespace

int64_t pairs_partial_doubles(int64_t n, int K)
{
    const int64_t items = pairs_items(n);
    const int64_t slots = K == 1 ? max_slots<1>() : K == 2 ? max_slots<2>() : max_slots<3>();
    // split items take four workgroups each
    return (pairs_split(items, slots) ? kPW * items : items) * 2 * (K + 1) * 3 * kPS;
}

int pairs_chunk(int64_t partial_cap, int K)
{
    const int64_t per_item = (int64_t)2 * (K + 1) * 3 * kPS;
    int cs = 64;
    while (cs > 0 && (int64_t)cs * cs * per_item > partial_cap) --cs;
    return cs;
}

hipError_t launch_force_pairs(const ForceArgs &a, Chain chain, hipStream_t st)
{
    if (a.n <= 0) return hipSuccess;
    if (a.k_first != 0 || a.K < 1 || a.K > 3) return hipErrorInvalidValue;
    const bool qm = a.qpart != nullptr;
    const bool single_fits = pairs_items(a.n) * 2 * (a.K + 1) * 3 * kPS <= a.partial_cap;
    if (a.n <= kPairsMaxN && (single_fits || !a.chunks_if_needed)) {
        // the whole items must fit (split ones only where they fit too)
        if (!single_fits) return hipErrorInvalidValue;
    } else {
        // chunked: no fused rate; chunks of at least 16 super-blocks
        if (qm || pairs_chunk(a.partial_cap, a.K) < kPairsMinChunk) return hipErrorInvalidValue;
    }
    if (qm && pairs_items(a.n) > a.qpart_cap) return hipErrorInvalidValue;
    switch (chain) {
        case Chain::Fp64: return qm ? launch_chain<Chain::Fp64, true>(a, st) : launch_chain<Chain::Fp64, false>(a, st);
        case Chain::Split:
            return qm ? launch_chain<Chain::Split, true>(a, st) : launch_chain<Chain::Split, false>(a, st);
        case Chain::Mixed:
            return qm ? launch_chain<Chain::Mixed, true>(a, st) : launch_chain<Chain::Mixed, false>(a, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hermite
