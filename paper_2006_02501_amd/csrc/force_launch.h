// Declarations of the O(N^2) evaluation: its chains, argument block, launch
// shapes and launcher (implemented in force_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hermite {

constexpr int kBlock = 256;   // threads per workgroup of the tiled evaluation (4 wave64)
constexpr int kTile = 256;    // j-particles staged in LDS per tile
constexpr int kMaxPath = 6;   // path derivatives x^(0..5) (generic initialisation)

enum class Chain { Fp64 = 0, Mixed = 1, Generic = 2, Split = 3 };

// Where the evaluation reads the j-particles from: LDS tiles filled by the
// workgroup, or packed records streamed through the scalar unit into SGPRs;
// or Pairs: every pair once, for both of its bodies (FP64, mixed and split
// chains, N <= kPairsMaxN; see launch_force_pairs).
enum class JSource { Lds = 0, Scalar = 1, Pairs = 2 };

struct ForceArgs {
    int64_t n;                    // particles (i and j range over all of them)
    const double *mass;           // [n]
    const double *path[kMaxPath]; // path[k] = [3][n] block of x^(k)
    int K;                        // highest derivative evaluated
    int k_first;                  // first derivative written (outputs k_first..K)
    double G, eps2;
    double *out;                  // [K+1-k_first][3][n]
    double *partial;              // split partial sums [nsplit][K+1-k_first][3][n]
    int64_t partial_cap;          // capacity of partial, in doubles
    double *jrec;                 // packed j-records [n][16] (scalar source)
    // Optional (FP64 and split chains): every workgroup also writes the
    // largest pair rate G (m_i + m_j) (r^2 + eps^2)^(-3/2) of its pairs to
    // qpart[block], and *q_count receives the number of workgroups.
    double *qpart = nullptr;
    int64_t qpart_cap = 0;
    int *q_count = nullptr;
    // Every-pair-once evaluation of at most kPairsMaxN bodies whose single
    // launch's partial sums exceed partial_cap: with this set it runs as
    // pairs of chunks sized to the workspace (as beyond kPairsMaxN) instead
    // of failing (no pair rate in that case).
    bool chunks_if_needed = false;
    // Evaluation of the i-particles [i_off, i_off + i_cnt) only, against every
    // j (one-sided kernels; i_cnt < 0: all n).  Outputs keep the [..][3][n]
    // layout; the other positions are not written.
    int64_t i_off = 0;
    int64_t i_cnt = -1;
};

// Launch shape of the FP64 / mixed evaluation (the generic initialisation
// chain always uses 4-wave workgroups with one i-particle per lane).
struct LaunchShape {
    int ipt;          // i-particles per lane: 1..4
    int waves;        // waves per workgroup: 4 or 16 (16 with ipt = 1 only)
    JSource jsource;  // LDS tiles, scalar stream, or every pair once
};

// Doubles per particle of the packed j-stream.
constexpr int kJRecDoubles = 16;

// Evaluates with the given chain, launch shape and j-split count.
hipError_t launch_force(const ForceArgs &a, Chain chain, const LaunchShape &shape, int nsplit, hipStream_t st);

// j-split count the evaluation uses when the caller does not fix one.
int auto_split(int64_t n, const LaunchShape &shape, bool generic);

// Every-pair-once evaluation (FP64, mixed or split chain, K = 1..3,
// k_first = 0): work items are pairs of 256-body super-blocks, each writing
// 2 * (K+1) * 3 * 256 partial sums into a.partial, which a fixed-order
// reduction adds into a.out.  Up to kPairsMaxN bodies one launch covers all
// pairs, with one workgroup per item and phase when the items are few
// (pairs_split) and a.partial (and a.qpart) hold them; with a.qpart it also
// writes one pair-rate maximum per workgroup (a.q_count = the workgroup
// count), from FP64 differences in every chain.
// Beyond kPairsMaxN the bodies are cut into chunks of pairs_chunk()
// super-blocks (at least kPairsMinChunk) and each chunk pair is one launch
// whose partials are added to the output in a fixed order (no rate).
constexpr int64_t kPairsMaxN = 32768;
constexpr int kPairsMinChunk = 16;
int64_t pairs_items(int64_t n);
// Items are split by phase when at most half as many as the `slots`
// workgroups the GPU holds at once.
bool pairs_split(int64_t items, int64_t slots);
// Partial sums a single launch may write, split items included (the device's
// resident-workgroup counts are queried on the current device).
int64_t pairs_partial_doubles(int64_t n, int K);
// Super-blocks per chunk whose rectangle of items fits partial_cap (<= 64).
int pairs_chunk(int64_t partial_cap, int K);
hipError_t launch_force_pairs(const ForceArgs &a, Chain chain, hipStream_t st);

}  // namespace hermite
