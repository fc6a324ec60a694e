// hermite_force_derivs_noalloc: the evaluation of hermite_force_derivs for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).  It takes no context:
// the every-pair-once evaluation's partial sums live in a file-scope device
// array of fixed size, one per GPU, held until the process ends, and the
// call allocates nothing on the host or the device.
#include "hermite.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>

#include "kernels.h"

namespace {

// 64 MiB of partial sums: one launch of the every-pair-once evaluation holds
// up to 13056 bodies at 8th order (15104 at 6th, 18688 at 4th); more bodies
// run as pairs of chunks sized to it (chunks of 36, 42 and 52 super-blocks
// of 256 bodies at 8th, 6th and 4th order).
constexpr int64_t kScratchDoubles = (int64_t)8 << 20;

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_scratch[kMaxDevices] = {};   // device address of scratch, per device

// Message of the calling thread's last failed call of this entry point.
thread_local char g_msg[256] = "";

hermite_status fail(hermite_status st, const char *msg)
{
    std::snprintf(g_msg, sizeof g_msg, "%s", msg);
    return st;
}

// The device address of this device's scratch array, looked up once per
// device with that device current (the array's name is a host-side stand-in
// and must never be passed to a kernel).
hermite_status scratch_ptr(double **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return fail(HERMITE_E_HIP, "hermite: no current HIP device (or more than 64 devices)");
    }
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(HERMITE_E_HIP, "hermite: hipGetSymbolAddress of the scratch array failed");
        }
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return HERMITE_OK;
}

}  // namespace

namespace hermite {
const char *noalloc_message() { return g_msg; }
}  // namespace hermite

extern "C" hermite_status hermite_force_derivs_noalloc(const hermite_params *prm, hermite_state *s, void *hip_stream)
{
    g_msg[0] = '\0';
    if (!prm) return fail(HERMITE_E_ARG, "hermite: params is NULL");
    if (prm->order != 4 && prm->order != 6 && prm->order != 8)
        return fail(HERMITE_E_ORDER, "hermite: order must be 4, 6 or 8");
    if (prm->precision != HERMITE_FP64 && prm->precision != HERMITE_MIXED && prm->precision != HERMITE_SPLIT)
        return fail(HERMITE_E_ARG, "hermite: precision must be HERMITE_FP64, HERMITE_MIXED or HERMITE_SPLIT");
    if (!std::isfinite(prm->G)) return fail(HERMITE_E_ARG, "hermite: G must be finite");
    if (!std::isfinite(prm->eps2) || prm->eps2 < 0.0) return fail(HERMITE_E_ARG, "hermite: eps2 must be finite and >= 0");
    if (!s) return fail(HERMITE_E_ARG, "hermite: state is NULL");
    if (s->n < 0 || s->n > ((int64_t)1 << 40)) return fail(HERMITE_E_ARG, "hermite: state n outside [0, 2^40]");
    if (s->n == 0) return HERMITE_OK;
    if (!s->mass || !s->pred || !s->eval) return fail(HERMITE_E_ARG, "hermite: state has a NULL mass/pred/eval pointer");
    const int p = prm->order / 2 - 1;
    // the smallest chunk the evaluation accepts must fit the scratch (it
    // does at every order: 16 x 16 items of at most 2 * 12 * 256 doubles)
    const int64_t per_item = (int64_t)2 * (p + 1) * 3 * 256;
    if ((int64_t)hermite::kPairsMinChunk * hermite::kPairsMinChunk * per_item > kScratchDoubles)
        return fail(HERMITE_E_ARG, "hermite: the static scratch cannot hold one chunk of the evaluation");
    double *ptr = nullptr;
    hermite_status st = scratch_ptr(&ptr);
    if (st != HERMITE_OK) return st;
    hermite::ForceArgs a{};
    a.n = s->n;
    a.mass = s->mass;
    const int64_t n3 = 3 * s->n;
    for (int k = 0; k <= p; ++k) a.path[k] = s->pred + k * n3;
    a.K = p;
    a.k_first = 0;
    a.G = prm->G;
    a.eps2 = prm->eps2;
    a.out = s->eval;
    a.partial = ptr;   // the device address, never the array's name
    a.partial_cap = kScratchDoubles;
    a.chunks_if_needed = true;
    const hermite::Chain chain = prm->precision == HERMITE_MIXED   ? hermite::Chain::Mixed
                                 : prm->precision == HERMITE_SPLIT ? hermite::Chain::Split
                                                                   : hermite::Chain::Fp64;
    const hipError_t e = hermite::launch_force_pairs(a, chain, (hipStream_t)hip_stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        char m[200];
        std::snprintf(m, sizeof m, "hermite: evaluation launch failed: %s", hipGetErrorString(e));
        return fail(HERMITE_E_HIP, m);
    }
    return HERMITE_OK;
}
