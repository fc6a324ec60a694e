// Host runtime behind include/hermite.h: argument validation, workspace,
// stream handling, launch-shape tuning, the P(EC)^n step sequence and the
// captured graph of the batched form.
#include "hermite.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"

using hermite::Chain;
using hermite::ForceArgs;

struct hermite_ctx {
    hermite_params prm{};
    int p = 1;
    int64_t n_max = 0;
    hipStream_t stream = nullptr;
    double *partial = nullptr;
    int64_t partial_cap = 0;
    int *flag = nullptr;
    int ipt = 1;
    int nsplit = 0;          // 0: automatic
    int jsource = 1;         // 0: LDS tiles, 1: scalar stream
    int waves = 4;           // waves per workgroup: 4 or 16
    double *jrec = nullptr;  // packed j-records [n_max][kJRecDoubles]
    // variable step: workgroup maxima of the pair rate, the device step
    // record (H_-, dt, H_+, failed) and its pinned host copy
    double *qpart = nullptr;
    int64_t qpart_cap = 0;
    double *vs = nullptr;
    double *host_vs = nullptr;
    std::string err;
    // batched form
    bool batch = false;
    int32_t n_sys = 0;
    int32_t n_bins = 0;
    int32_t max_size = 0;
    std::vector<int64_t> offsets;
    int32_t *d_bin_start = nullptr;
    int32_t *d_bin_sys = nullptr;
    int64_t *d_offsets = nullptr;
    int *d_counter = nullptr;
    int32_t *d_iters = nullptr;   // per-system iteration counts [n_sys]
    int32_t *h_iters = nullptr;   // their pinned staging copy
    hipEvent_t iters_copied = nullptr;   // recorded after the staging copy is enqueued
    // ensemble form
    bool ensemble = false;
    hermite::EnsembleCfg *d_cfg = nullptr;
    hermite::EnsembleStatus *d_status = nullptr;
    int cus = 256;                                 // compute units of the device (batched form)
    hermite::BatchShape bshape{1280, 1, 57};   // launch shape of the batched run (set at creation)
    bool bshape_set = false;                       // fixed by hermite_batch_set_launch or the autotuner
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    struct Key {
        const double *mass, *dt;
        double *pos, *vel, *deriv, *comp;
        int n_steps, n_iter;
        hermite::BatchShape shape;
        bool per_system;
        bool operator==(const Key &o) const
        {
            return mass == o.mass && dt == o.dt && pos == o.pos && vel == o.vel && deriv == o.deriv &&
                   comp == o.comp && n_steps == o.n_steps && n_iter == o.n_iter &&
                   shape.workgroups == o.shape.workgroups && shape.waves == o.shape.waves &&
                   shape.ring_min == o.shape.ring_min && per_system == o.per_system;
        }
    } key{};
};

namespace {

const char *kNoCtxMsg = "hermite: null context";

// Largest n_max accepted: keeps every workspace size (at most a few hundred
// bytes per body) far from 64-bit overflow.
constexpr int64_t kMaxBodies = (int64_t)1 << 40;

hermite_status fail(hermite_ctx *ctx, hermite_status st, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return st;
}

// A failed HIP call also leaves its code in the runtime's per-thread
// last-error slot, where the caller's next error check (torch's, say) would
// find it; the library reports through its own status instead, so it clears it.
void clear_hip_error() { (void)hipGetLastError(); }

hermite_status hip_fail(hermite_ctx *ctx, hipError_t e, const char *where)
{
    clear_hip_error();
    std::string m = std::string("hermite: HIP error in ") + where + ": " + hipGetErrorString(e);
    return fail(ctx, HERMITE_E_HIP, m);
}

#define HIP_TRY(ctx, expr, where)                  \
    do {                                           \
        hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, where); \
    } while (0)

hermite_status check_params(const hermite_params *prm, std::string &msg)
{
    if (!prm) { msg = "hermite: params is NULL"; return HERMITE_E_ARG; }
    if (prm->order != 4 && prm->order != 6 && prm->order != 8) {
        msg = "hermite: order must be 4, 6 or 8";
        return HERMITE_E_ORDER;
    }
    if (prm->precision != HERMITE_FP64 && prm->precision != HERMITE_MIXED && prm->precision != HERMITE_SPLIT) {
        msg = "hermite: precision must be HERMITE_FP64, HERMITE_MIXED or HERMITE_SPLIT";
        return HERMITE_E_ARG;
    }
    if (prm->corrector < 0 || prm->corrector > 2) { msg = "hermite: unknown corrector"; return HERMITE_E_ARG; }
    if (!std::isfinite(prm->G)) { msg = "hermite: G must be finite"; return HERMITE_E_ARG; }
    if (!std::isfinite(prm->eps2) || prm->eps2 < 0.0) { msg = "hermite: eps2 must be finite and >= 0"; return HERMITE_E_ARG; }
    if (prm->compensated != 0 && prm->compensated != 1) { msg = "hermite: compensated must be 0 or 1"; return HERMITE_E_ARG; }
    return HERMITE_OK;
}

hermite_status check_state(hermite_ctx *ctx, const hermite_state *s, bool need_init, bool need_pred_eval)
{
    if (!ctx) return HERMITE_E_ARG;
    if (!s) return fail(ctx, HERMITE_E_ARG, "hermite: state is NULL");
    if (s->n < 0 || s->n > ctx->n_max) return fail(ctx, HERMITE_E_ARG, "hermite: state n outside [0, n_max]");
    if (s->n > 0) {
        if (!s->mass || !s->pos || !s->vel || !s->deriv)
            return fail(ctx, HERMITE_E_ARG, "hermite: state has a NULL mass/pos/vel/deriv pointer");
        if (need_pred_eval && (!s->pred || !s->eval))
            return fail(ctx, HERMITE_E_ARG, "hermite: state has a NULL pred/eval pointer");
        if (ctx->prm.compensated && !s->comp)
            return fail(ctx, HERMITE_E_ARG, "hermite: compensated summation needs the state's comp array");
    }
    if (need_init && !s->initialized) return fail(ctx, HERMITE_E_STATE, "hermite: state not initialised (hermite_init)");
    return HERMITE_OK;
}

bool good_dt(double dt) { return std::isfinite(dt) && dt != 0.0; }

// t advances by dt: plainly, or by compensated summation with the state's
// t_comp (the same rule the corrector applies to x and v).
void advance_time(const hermite_ctx *ctx, hermite_state *s, double dt)
{
    if (!ctx->prm.compensated) {
        s->t += dt;
        return;
    }
    const double y = dt - s->t_comp;
    const double t1 = s->t + y;
    s->t_comp = (t1 - s->t) - y;
    s->t = t1;
}

double *comp_of(const hermite_ctx *ctx, hermite_state *s) { return ctx->prm.compensated ? s->comp : nullptr; }

int64_t partial_capacity(int64_t n_max, int p)
{
    // Split partial sums of up to p+1 derivative blocks.  Enough for every
    // split count the launch tuning may pick: up to 64 splits while
    // n * splits stays below ~4 Mi, at least 4 splits at any n <= n_max.
    if (n_max <= 0) return 0;
    const int64_t nv = p + 1;
    int64_t ns = ((int64_t)4 << 20) / n_max;
    ns = std::max<int64_t>(4, std::min<int64_t>(64, ns));
    int64_t cap = nv * 3 * n_max * ns;
    // and the every-pair-once partials (at most 2 * 12 * 256 doubles for each
    // of the ~n^2 / 131072 super-block pairs)
    if (n_max <= hermite::kPairsMaxN) cap = std::max(cap, hermite::pairs_partial_doubles(n_max, p));
    return cap;
}

// The every-pair-once evaluation of n bodies fits this context's workspace:
// in one launch up to kPairsMaxN bodies, in chunks beyond.
bool pairs_fit(const hermite_ctx *ctx, int64_t n)
{
    if (n <= hermite::kPairsMaxN)
        return hermite::pairs_partial_doubles(n, ctx->p) <= ctx->partial_cap &&
               hermite::pairs_items(n) <= ctx->qpart_cap;
    return hermite::pairs_chunk(ctx->partial_cap, ctx->p) >= hermite::kPairsMinChunk;
}

// The every-pair-once evaluation of n bodies takes the step criterion's rate
// along (one launch; the chunked form does not).
bool pairs_rate(int64_t n) { return n <= hermite::kPairsMaxN; }

hermite_status run_force(hermite_ctx *ctx, const hermite_state *s, Chain chain, int K, int k_first,
                         const double *const *path, double *out, int ipt, int nsplit, int jsource, int waves,
                         int *q_count = nullptr, int64_t i0 = 0, int64_t ni = -1)
{
    ForceArgs a{};
    a.n = s->n;
    a.i_off = i0;
    a.i_cnt = ni;
    a.mass = s->mass;
    for (int k = 0; k <= K; ++k) a.path[k] = path[k];
    a.K = K;
    a.k_first = k_first;
    a.G = ctx->prm.G;
    a.eps2 = ctx->prm.eps2;
    a.out = out;
    a.partial = ctx->partial;
    a.partial_cap = ctx->partial_cap;
    a.jrec = ctx->jrec;
    if (q_count) {
        a.qpart = ctx->qpart;
        a.qpart_cap = ctx->qpart_cap;
        a.q_count = q_count;
    }
    const hermite::JSource src = jsource == 2 ? hermite::JSource::Pairs
                                 : jsource == 1 ? hermite::JSource::Scalar
                                                : hermite::JSource::Lds;
    hermite::LaunchShape sh{ipt, waves, src};
    if (src == hermite::JSource::Pairs && (chain == Chain::Generic || !pairs_fit(ctx, s->n)))
        return fail(ctx, HERMITE_E_ARG, "hermite: the every-pair-once evaluation does not fit this context's workspace");
    if (nsplit <= 0) nsplit = hermite::auto_split(ni >= 0 ? ni : s->n, sh, chain == Chain::Generic);
    HIP_TRY(ctx, hermite::launch_force(a, chain, sh, nsplit, ctx->stream), "force kernel launch");
    return HERMITE_OK;
}

hermite_status check_finite(hermite_ctx *ctx, const double *const *arrays, const int64_t *counts, int narr)
{
    HIP_TRY(ctx, hipMemsetAsync(ctx->flag, 0, sizeof(int), ctx->stream), "finite-flag clear");
    for (int i = 0; i < narr; ++i)
        HIP_TRY(ctx, hermite::launch_check_finite(arrays[i], counts[i], ctx->flag, ctx->stream), "finite check");
    int h = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&h, ctx->flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream), "finite-flag copy");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "finite-flag sync");
    if (h) return fail(ctx, HERMITE_E_NONFINITE, "hermite: non-finite value in the state");
    return HERMITE_OK;
}

hermite_status alloc_timestep(hermite_ctx *ctx)
{
    // the rate pass writes at most min(ceil(n/256) ceil(n/128), ceil(n/256) +
    // 8191) workgroup maxima, which is at most n rounded up to 64;
    // an evaluation with the fused rate at most one per workgroup, i.e. at
    // most (ceil(n/64)) * 64 splits
    ctx->qpart_cap = std::max<int64_t>((ctx->n_max + 255) / 256 + 4097, (ctx->n_max + 63) / 64 * 64);
    if (hipMalloc((void **)&ctx->qpart, ctx->qpart_cap * sizeof(double)) != hipSuccess) return HERMITE_E_ALLOC;
    if (hipMalloc((void **)&ctx->vs, hermite::kVsLen * sizeof(double)) != hipSuccess) return HERMITE_E_ALLOC;
    if (hipHostMalloc((void **)&ctx->host_vs, hermite::kVsLen * sizeof(double), hipHostMallocDefault) != hipSuccess)
        return HERMITE_E_ALLOC;
    return HERMITE_OK;
}

void free_ctx(hermite_ctx *ctx)
{
    if (!ctx) return;
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    if (ctx->partial) (void)hipFree(ctx->partial);
    if (ctx->flag) (void)hipFree(ctx->flag);
    if (ctx->d_bin_start) (void)hipFree(ctx->d_bin_start);
    if (ctx->d_bin_sys) (void)hipFree(ctx->d_bin_sys);
    if (ctx->d_offsets) (void)hipFree(ctx->d_offsets);
    if (ctx->d_counter) (void)hipFree(ctx->d_counter);
    if (ctx->d_iters) (void)hipFree(ctx->d_iters);
    if (ctx->h_iters) (void)hipHostFree(ctx->h_iters);
    if (ctx->iters_copied) (void)hipEventDestroy(ctx->iters_copied);
    if (ctx->d_cfg) (void)hipFree(ctx->d_cfg);
    if (ctx->d_status) (void)hipFree(ctx->d_status);
    if (ctx->jrec) (void)hipFree(ctx->jrec);
    if (ctx->qpart) (void)hipFree(ctx->qpart);
    if (ctx->vs) (void)hipFree(ctx->vs);
    if (ctx->host_vs) (void)hipHostFree(ctx->host_vs);
    delete ctx;
}

hermite_status alloc_failed(hermite_ctx *ctx)
{
    clear_hip_error();
    free_ctx(ctx);
    return HERMITE_E_ALLOC;
}

Chain eval_chain(const hermite_ctx *ctx)
{
    return ctx->prm.precision == HERMITE_MIXED ? Chain::Mixed
           : ctx->prm.precision == HERMITE_SPLIT ? Chain::Split
                                                 : Chain::Fp64;
}

// One evaluation of the current path; with q_count, the pair rate is taken
// along (FP64 and split chains) and the workgroup maxima land in ctx->qpart.
hermite_status eval_path(hermite_ctx *ctx, hermite_state *s, int *q_count)
{
    const int p = ctx->p;
    const int64_t n3 = 3 * s->n;
    const double *path[hermite::kMaxPath] = {};
    for (int k = 0; k <= p; ++k) path[k] = s->pred + k * n3;
    return run_force(ctx, s, eval_chain(ctx), p, 0, path, s->eval, ctx->ipt, ctx->nsplit, ctx->jsource, ctx->waves,
                     q_count);
}

// Launch-shape tuning cache: the autotuners' picks, keyed by what the best
// shape depends on (the evaluation or the batched run, order, precision, the
// problem size or the histogram of system sizes, the device's architecture
// and CU count).  Kept for the life of the process; when the environment
// variable HERMITE_TUNE_CACHE names a file, entries are also read from it at
// first use and appended to it (one "key<TAB>values" line each).
class TuneCache {
public:
    bool get(const std::string &key, std::vector<int> &val)
    {
        std::lock_guard<std::mutex> g(mu_);
        load();
        auto it = map_.find(key);
        if (it == map_.end()) return false;
        val = it->second;
        return true;
    }
    void put(const std::string &key, const std::vector<int> &val)
    {
        std::lock_guard<std::mutex> g(mu_);
        load();
        map_[key] = val;
        const char *path = std::getenv("HERMITE_TUNE_CACHE");
        if (!path || !*path) return;
        if (FILE *f = std::fopen(path, "a")) {
            std::fprintf(f, "%s\t", key.c_str());
            for (size_t i = 0; i < val.size(); ++i) std::fprintf(f, i ? " %d" : "%d", val[i]);
            std::fprintf(f, "\n");
            std::fclose(f);
        }
    }
    void clear()
    {
        std::lock_guard<std::mutex> g(mu_);
        map_.clear();
        loaded_ = true;   // a cleared cache does not re-read the file
    }

private:
    void load()
    {
        if (loaded_) return;
        loaded_ = true;
        const char *path = std::getenv("HERMITE_TUNE_CACHE");
        if (!path || !*path) return;
        FILE *f = std::fopen(path, "r");
        if (!f) return;
        char line[1024];
        while (std::fgets(line, sizeof line, f)) {
            char *tab = std::strchr(line, '\t');
            if (!tab) continue;
            std::string key(line, tab);
            std::vector<int> val;
            char *p = tab + 1;
            for (;;) {
                char *end = nullptr;
                const long x = std::strtol(p, &end, 10);
                if (end == p) break;
                val.push_back((int)x);
                p = end;
            }
            if (!val.empty()) map_[key] = val;
        }
        std::fclose(f);
    }
    std::mutex mu_;
    std::map<std::string, std::vector<int>> map_;
    bool loaded_ = false;
};

TuneCache &tune_cache()
{
    static TuneCache c;
    return c;
}

// Architecture name and CU count of the current device, for cache keys.
std::string device_tag()
{
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        clear_hip_error();
        return "unknown";
    }
    char buf[320];
    std::snprintf(buf, sizeof buf, "%s:%d", prop.gcnArchName, prop.multiProcessorCount);
    return buf;
}

// Workgroups of a batched shape that the device holds at once.
int batch_resident(const hermite_ctx *ctx, const hermite::BatchShape &sh)
{
    const int per_cu = hermite::batch_resident_per_cu(sh, ctx->p, ctx->prm.precision == HERMITE_MIXED,
                                                      ctx->prm.compensated != 0);
    if (per_cu <= 0) clear_hip_error();
    return std::max(1, per_cu) * ctx->cus;
}

// Default batched shape: two waves per bin, the whole-wave ring from 57
// bodies, and as many persistent workgroups as the GPU holds (the fastest
// shape on the 4096-system workload, in both chains).  Systems of at most 16
// bodies take at most 8 sweep steps, too few to share: one wave.  A batch
// whose bins all fit on the GPU at once with four waves each takes four: a
// bin's time then sets the run's, and four waves split its sweep further
// (one 64-body system, 4th order: 4.0 against 7.4 us per step).
hermite::BatchShape default_batch_shape(const hermite_ctx *ctx)
{
    int waves = ctx->max_size <= 16 ? 1 : 2;
    if (waves == 2 && ctx->n_bins <= batch_resident(ctx, hermite::BatchShape{0, 4, 57})) waves = 4;
    hermite::BatchShape sh{0, waves, 57};
    sh.workgroups = batch_resident(ctx, sh);
    return sh;
}

}  // namespace

extern "C" {

const char *hermite_version(void) { return "paper_2006_02501_amd hermite 0.1 (gfx950)"; }

const char *hermite_last_error(const hermite_ctx *ctx)
{
    if (ctx) return ctx->err.c_str();
    const char *m = hermite::noalloc_message();
    return m && *m ? m : kNoCtxMsg;
}

hermite_status hermite_create(const hermite_params *prm, int64_t n_max, void *hip_stream, hermite_ctx **out)
{
    std::string msg;
    if (!out) return HERMITE_E_ARG;
    *out = nullptr;
    hermite_status st = check_params(prm, msg);
    if (st != HERMITE_OK) return st;
    if (n_max < 0 || n_max > kMaxBodies) return HERMITE_E_ARG;
    hermite_ctx *ctx = new hermite_ctx();
    ctx->prm = *prm;
    ctx->p = prm->order / 2 - 1;
    ctx->n_max = n_max;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->partial_cap = partial_capacity(n_max, ctx->p);
    if (ctx->partial_cap > 0 && hipMalloc((void **)&ctx->partial, ctx->partial_cap * sizeof(double)) != hipSuccess) {
        return alloc_failed(ctx);
    }
    if (hipMalloc((void **)&ctx->flag, sizeof(int)) != hipSuccess) {
        return alloc_failed(ctx);
    }
    if (n_max > 0 &&
        hipMalloc((void **)&ctx->jrec, (size_t)n_max * hermite::kJRecDoubles * sizeof(double)) != hipSuccess) {
        return alloc_failed(ctx);
    }
    if (alloc_timestep(ctx) != HERMITE_OK) {
        return alloc_failed(ctx);
    }
    *out = ctx;
    return HERMITE_OK;
}

hermite_status hermite_destroy(hermite_ctx *ctx)
{
    free_ctx(ctx);
    return HERMITE_OK;
}

hermite_status hermite_set_stream(hermite_ctx *ctx, void *hip_stream)
{
    if (!ctx) return HERMITE_E_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return HERMITE_OK;
}

hermite_status hermite_set_launch(hermite_ctx *ctx, int32_t i_per_thread, int32_t j_split, int32_t j_source,
                                  int32_t wg_waves)
{
    if (!ctx) return HERMITE_E_ARG;
    if (i_per_thread < 1 || i_per_thread > 4)
        return fail(ctx, HERMITE_E_ARG, "hermite: i_per_thread must be 1, 2, 3 or 4");
    if (i_per_thread > 2 && (j_source != 1 || wg_waves != 4))
        return fail(ctx, HERMITE_E_ARG,
                    "hermite: 3 or 4 i-particles per lane need the scalar j-source and 4-wave workgroups");
    if (j_split < 0 || j_split > 64) return fail(ctx, HERMITE_E_ARG, "hermite: j_split must be in 0..64");
    if (j_source < 0 || j_source > 2) return fail(ctx, HERMITE_E_ARG, "hermite: j_source must be 0, 1 or 2");
    if (j_source == 2 && (i_per_thread != 1 || wg_waves != 4))
        return fail(ctx, HERMITE_E_ARG,
                    "hermite: the every-pair-once evaluation (j_source 2) takes one i-particle per lane and "
                    "4-wave workgroups");
    if (wg_waves != 4 && wg_waves != 16) return fail(ctx, HERMITE_E_ARG, "hermite: wg_waves must be 4 or 16");
    if (wg_waves == 16 && (i_per_thread != 1 || j_source != 1))
        return fail(ctx, HERMITE_E_ARG,
                    "hermite: 16-wave workgroups take one i-particle per lane and the scalar j-source");
    ctx->ipt = i_per_thread;
    ctx->nsplit = j_split;
    ctx->jsource = j_source;
    ctx->waves = wg_waves;
    return HERMITE_OK;
}

hermite_status hermite_init(hermite_ctx *ctx, hermite_state *s)
{
    if (!ctx) return HERMITE_E_ARG;
    if (ctx->batch || ctx->ensemble)
        return fail(ctx, HERMITE_E_ARG, "hermite: batched or ensemble context, use its own init");
    hermite_status st = check_state(ctx, s, false, false);
    if (st != HERMITE_OK) return st;
    const int p = ctx->p;
    const int64_t n3 = 3 * s->n;
    if (ctx->prm.compensated) {
        s->t_comp = 0.0;
        if (s->n > 0)
            HIP_TRY(ctx, hipMemsetAsync(s->comp, 0, (size_t)2 * n3 * sizeof(double), ctx->stream), "comp clear");
    }
    if (s->n > 0) {
        // pass 1: a, adot from (x, v)
        const double *path[hermite::kMaxPath] = {s->pos, s->vel};
        st = run_force(ctx, s, Chain::Generic, 1, 0, path, s->deriv, 1, 0, 0, 4);
        if (st != HERMITE_OK) return st;
        if (p >= 2) {   // pass 2: a^(2), a^(3) from (x, v, a, adot)
            const double *path2[hermite::kMaxPath] = {s->pos, s->vel, s->deriv, s->deriv + n3};
            st = run_force(ctx, s, Chain::Generic, 3, 2, path2, s->deriv + 2 * n3, 1, 0, 0, 4);
            if (st != HERMITE_OK) return st;
        }
        if (p >= 3) {   // pass 3: a^(4), a^(5) from (x, v, a, ..., a^(3))
            const double *path3[hermite::kMaxPath] = {s->pos, s->vel, s->deriv, s->deriv + n3,
                                                      s->deriv + 2 * n3, s->deriv + 3 * n3};
            st = run_force(ctx, s, Chain::Generic, 5, 4, path3, s->deriv + 4 * n3, 1, 0, 0, 4);
            if (st != HERMITE_OK) return st;
        }
    }
    s->initialized = 1;
    return HERMITE_OK;
}

hermite_status hermite_predict(hermite_ctx *ctx, hermite_state *s, double dt)
{
    if (!ctx) return HERMITE_E_ARG;
    if (ctx->batch || ctx->ensemble) return fail(ctx, HERMITE_E_ARG, "hermite: batched or ensemble context");
    if (!good_dt(dt)) return fail(ctx, HERMITE_E_ARG, "hermite: dt must be finite and nonzero");
    hermite_status st = check_state(ctx, s, true, true);
    if (st != HERMITE_OK) return st;
    HIP_TRY(ctx, hermite::launch_predict(ctx->p, s->n, dt, nullptr, s->pos, s->vel, s->deriv, s->pred, ctx->stream),
            "predict launch");
    return HERMITE_OK;
}

hermite_status hermite_force_derivs(hermite_ctx *ctx, hermite_state *s)
{
    if (!ctx) return HERMITE_E_ARG;
    if (ctx->batch || ctx->ensemble) return fail(ctx, HERMITE_E_ARG, "hermite: batched or ensemble context");
    hermite_status st = check_state(ctx, s, false, true);
    if (st != HERMITE_OK) return st;
    return eval_path(ctx, s, nullptr);
}

hermite_status hermite_force_derivs_range(hermite_ctx *ctx, hermite_state *s, int64_t i0, int64_t ni)
{
    if (!ctx) return HERMITE_E_ARG;
    if (ctx->batch || ctx->ensemble) return fail(ctx, HERMITE_E_ARG, "hermite: batched or ensemble context");
    hermite_status st = check_state(ctx, s, false, true);
    if (st != HERMITE_OK) return st;
    if (i0 < 0 || ni < 0 || i0 > s->n || ni > s->n - i0)
        return fail(ctx, HERMITE_E_ARG, "hermite: i-range outside [0, n)");
    if (ni == 0) return HERMITE_OK;
    // the context's one-sided launch shape; every pair once has no one-sided
    // form, so that choice takes the LDS source with two i-particles per lane
    // (FP64, split) or the scalar source with one (mixed)
    int ipt = ctx->ipt, jsource = ctx->jsource, waves = ctx->waves, nsplit = ctx->nsplit;
    if (jsource == 2) {
        const bool mixed = ctx->prm.precision == HERMITE_MIXED;
        ipt = mixed ? 1 : 2;
        jsource = mixed ? 1 : 0;
        waves = 4;
        nsplit = 0;
    }
    const int p = ctx->p;
    const int64_t n3 = 3 * s->n;
    const double *path[hermite::kMaxPath] = {};
    for (int k = 0; k <= p; ++k) path[k] = s->pred + k * n3;
    return run_force(ctx, s, eval_chain(ctx), p, 0, path, s->eval, ipt, nsplit, jsource, waves, nullptr, i0, ni);
}

hermite_status hermite_correct(hermite_ctx *ctx, hermite_state *s, double dt, int32_t last_iter)
{
    if (!ctx) return HERMITE_E_ARG;
    if (ctx->batch || ctx->ensemble) return fail(ctx, HERMITE_E_ARG, "hermite: batched or ensemble context");
    if (!good_dt(dt)) return fail(ctx, HERMITE_E_ARG, "hermite: dt must be finite and nonzero");
    hermite_status st = check_state(ctx, s, true, true);
    if (st != HERMITE_OK) return st;
    HIP_TRY(ctx, hermite::launch_correct(ctx->p, ctx->prm.corrector, last_iter ? 1 : 0, s->n, dt, nullptr, nullptr,
                                         s->pos, s->vel, s->deriv, s->eval, s->pred, comp_of(ctx, s), ctx->stream),
            "correct launch");
    if (last_iter) advance_time(ctx, s, dt);
    return HERMITE_OK;
}

hermite_status hermite_step(hermite_ctx *ctx, hermite_state *s, double dt, int32_t n_iter)
{
    if (!ctx) return HERMITE_E_ARG;
    if (ctx->batch || ctx->ensemble)
        return fail(ctx, HERMITE_E_ARG, "hermite: batched or ensemble context, use its own run call");
    if (n_iter < 1) return fail(ctx, HERMITE_E_ARG, "hermite: n_iter must be >= 1");
    if (!good_dt(dt)) return fail(ctx, HERMITE_E_ARG, "hermite: dt must be finite and nonzero");
    hermite_status st = check_state(ctx, s, true, true);
    if (st != HERMITE_OK) return st;
    st = hermite_predict(ctx, s, dt);
    for (int it = 0; it < n_iter && st == HERMITE_OK; ++it) {
        st = hermite_force_derivs(ctx, s);
        if (st == HERMITE_OK) st = hermite_correct(ctx, s, dt, it == n_iter - 1);
    }
    if (st != HERMITE_OK || !ctx->prm.check_finite || s->n == 0) return st;
    const double *arrs[3] = {s->pos, s->vel, s->deriv};
    const int64_t cnt[3] = {3 * s->n, 3 * s->n, (int64_t)2 * ctx->p * 3 * s->n};
    return check_finite(ctx, arrs, cnt, 3);
}

hermite_status hermite_step_criterion(hermite_ctx *ctx, const hermite_state *s, double eta, double *h)
{
    if (!ctx) return HERMITE_E_ARG;
    if (ctx->batch || ctx->ensemble) return fail(ctx, HERMITE_E_ARG, "hermite: batched or ensemble context");
    hermite_status st = check_state(ctx, s, false, false);
    if (st != HERMITE_OK) return st;
    if (!h) return fail(ctx, HERMITE_E_ARG, "hermite: h is NULL");
    if (!std::isfinite(eta) || !(eta > 0.0)) return fail(ctx, HERMITE_E_ARG, "hermite: eta must be finite and > 0");
    if (s->n < 2) return fail(ctx, HERMITE_E_ARG, "hermite: the step criterion needs at least two particles");
    HIP_TRY(ctx, hermite::launch_timestep(s->n, s->mass, s->pos, ctx->prm.G, ctx->prm.eps2, eta, 1.0, 0, 1,
                                          ctx->qpart, ctx->qpart_cap, ctx->vs, ctx->stream),
            "step criterion launch");
    HIP_TRY(ctx, hipMemcpyAsync(ctx->host_vs, ctx->vs, hermite::kVsLen * sizeof(double), hipMemcpyDeviceToHost,
                                ctx->stream),
            "step criterion copy");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "step criterion sync");
    *h = ctx->host_vs[0];
    if (ctx->host_vs[3] != 0.0)
        return fail(ctx, HERMITE_E_NONFINITE,
                    "hermite: step criterion not finite and positive (no pair with G (m_i + m_j) > 0, "
                    "coincident bodies without softening, or non-finite positions)");
    return HERMITE_OK;
}

hermite_status hermite_step_symmetric(hermite_ctx *ctx, hermite_state *s, double eta, int32_t n_iter,
                                      double direction, double *dt_taken)
{
    if (!ctx) return HERMITE_E_ARG;
    if (ctx->batch || ctx->ensemble) return fail(ctx, HERMITE_E_ARG, "hermite: batched or ensemble context");
    if (n_iter < 1) return fail(ctx, HERMITE_E_ARG, "hermite: n_iter must be >= 1");
    if (!std::isfinite(eta) || !(eta > 0.0)) return fail(ctx, HERMITE_E_ARG, "hermite: eta must be finite and > 0");
    if (direction != 1.0 && direction != -1.0) return fail(ctx, HERMITE_E_ARG, "hermite: direction must be +1 or -1");
    hermite_status st = check_state(ctx, s, true, true);
    if (st != HERMITE_OK) return st;
    if (s->n < 2) return fail(ctx, HERMITE_E_ARG, "hermite: the step criterion needs at least two particles");
    const int p = ctx->p;
    // The step length alternates between the device slots vs[1] and vs[4]:
    // an iteration corrects with the one its path was formed for while the
    // criterion at its evaluation point writes the next one into the other.
    double *vs = ctx->vs;
    // H_- at the start, a first prediction with dt = s H_-, H_+ at its end
    // point, and the prediction for dt = s (H_- + H_+)/2
    HIP_TRY(ctx, hermite::launch_timestep(s->n, s->mass, s->pos, ctx->prm.G, ctx->prm.eps2, eta, direction, 0, 1,
                                          ctx->qpart, ctx->qpart_cap, vs, ctx->stream),
            "step criterion launch");
    HIP_TRY(ctx, hermite::launch_predict(p, s->n, 0.0, vs + 1, s->pos, s->vel, s->deriv, s->pred, ctx->stream),
            "predict launch");
    HIP_TRY(ctx, hermite::launch_timestep(s->n, s->mass, s->pred, ctx->prm.G, ctx->prm.eps2, eta, direction, 1, 4,
                                          ctx->qpart, ctx->qpart_cap, vs, ctx->stream),
            "step criterion launch");
    HIP_TRY(ctx, hermite::launch_predict(p, s->n, 0.0, vs + 4, s->pos, s->vel, s->deriv, s->pred, ctx->stream),
            "predict launch");
    // FP64 and split evaluations take the pair rate along, and so does the
    // mixed every-pair-once evaluation (from its FP64 differences) while it is
    // one launch; the other mixed kernels have only an FP32 1/r and the
    // chunked every-pair-once form keeps no rate, so their criterion is a
    // separate FP64 pass
    const bool pairs = ctx->jsource == 2;
    const bool fused = pairs ? pairs_rate(s->n) : ctx->prm.precision != HERMITE_MIXED;
    int cur = 4, nxt = 1;
    for (int it = 0; it < n_iter; ++it) {
        const bool last = it == n_iter - 1;
        // evaluation at t0 + dt; before the last iteration also H_+ at this
        // evaluation point, and from it the next dt = s (H_- + H_+)/2
        if (last) {
            st = eval_path(ctx, s, nullptr);
            if (st != HERMITE_OK) return st;
        } else if (fused) {
            int nq = 0;
            st = eval_path(ctx, s, &nq);
            if (st != HERMITE_OK) return st;
            HIP_TRY(ctx, hermite::launch_timestep_fold(ctx->qpart, nq, eta, direction, 1, nxt, vs, ctx->stream),
                    "step criterion launch");
        } else {
            st = eval_path(ctx, s, nullptr);
            if (st != HERMITE_OK) return st;
            HIP_TRY(ctx, hermite::launch_timestep(s->n, s->mass, s->pred, ctx->prm.G, ctx->prm.eps2, eta, direction,
                                                  1, nxt, ctx->qpart, ctx->qpart_cap, vs, ctx->stream),
                    "step criterion launch");
        }
        // correction with this iteration's dt; before the last iteration the
        // iterate, moved to t0 + next dt, is the next path
        HIP_TRY(ctx, hermite::launch_correct(p, ctx->prm.corrector, last ? 1 : 0, s->n, 0.0, vs + cur,
                                             last ? nullptr : vs + nxt, s->pos, s->vel, s->deriv, s->eval, s->pred,
                                             comp_of(ctx, s), ctx->stream),
                "correct launch");
        if (!last) std::swap(cur, nxt);
    }
    HIP_TRY(ctx, hipMemcpyAsync(ctx->host_vs, vs, hermite::kVsLen * sizeof(double), hipMemcpyDeviceToHost,
                                ctx->stream),
            "step length copy");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "step length sync");
    if (ctx->host_vs[3] != 0.0)
        return fail(ctx, HERMITE_E_NONFINITE,
                    "hermite: step criterion not finite and positive (no pair with G (m_i + m_j) > 0, "
                    "coincident bodies without softening, or non-finite positions); state unchanged");
    const double dt = ctx->host_vs[cur];
    advance_time(ctx, s, dt);
    if (dt_taken) *dt_taken = dt;
    if (!ctx->prm.check_finite) return HERMITE_OK;
    const double *arrs[3] = {s->pos, s->vel, s->deriv};
    const int64_t cnt[3] = {3 * s->n, 3 * s->n, (int64_t)2 * p * 3 * s->n};
    return check_finite(ctx, arrs, cnt, 3);
}

hermite_status hermite_potential(hermite_ctx *ctx, const hermite_state *s, double *phi)
{
    if (!ctx) return HERMITE_E_ARG;
    if (ctx->batch || ctx->ensemble) return fail(ctx, HERMITE_E_ARG, "hermite: batched or ensemble context");
    hermite_status st = check_state(ctx, s, false, false);
    if (st != HERMITE_OK) return st;
    if (s->n > 0 && !phi) return fail(ctx, HERMITE_E_ARG, "hermite: phi is NULL");
    HIP_TRY(ctx, hermite::launch_potential(s->n, s->mass, s->pos, ctx->prm.G, ctx->prm.eps2, phi, ctx->stream),
            "potential launch");
    return HERMITE_OK;
}

hermite_status hermite_autotune(hermite_ctx *ctx, hermite_state *s, int32_t *i_per_thread, int32_t *j_split,
                                int32_t *j_source, int32_t *wg_waves)
{
    if (!ctx) return HERMITE_E_ARG;
    if (ctx->batch || ctx->ensemble) return fail(ctx, HERMITE_E_ARG, "hermite: batched or ensemble context");
    hermite_status st = check_state(ctx, s, false, true);
    if (st != HERMITE_OK) return st;
    struct Cand {
        int ipt, waves, src;
    };
    struct Timed {
        Cand c;
        int split;
        float ms;
        int64_t partials;   // partial sums the shape writes per evaluation (doubles)
    };
    const Cand shapes[] = {{1, 4, 0}, {2, 4, 0}, {1, 4, 1}, {2, 4, 1}, {3, 4, 1}, {4, 4, 1}, {1, 16, 1}, {1, 4, 2}};
    int best_ipt = 1, best_split = 0, best_src = 1, best_waves = 4;
    // cache key: order, precision, the size bucket (a quarter octave of n) and the device
    char key[384];
    std::snprintf(key, sizeof key, "force|p=%d|prec=%d|nb=%d|dev=%s", ctx->p, ctx->prm.precision,
                  s->n > 0 ? (int)std::floor(4.0 * std::log2((double)s->n)) : -1, device_tag().c_str());
    std::vector<int> cached;
    bool hit = false;
    if (s->n > 0 && tune_cache().get(key, cached) && cached.size() == 4) {
        // a cached shape is taken only if this context can run it
        const bool pairs_ok = cached[2] != 2 || pairs_fit(ctx, s->n);
        if (pairs_ok && hermite_set_launch(ctx, cached[0], cached[1], cached[2], cached[3]) == HERMITE_OK) {
            best_ipt = cached[0];
            best_split = cached[1];
            best_src = cached[2];
            best_waves = cached[3];
            hit = true;
        }
    }
    if (s->n > 0 && !hit) {
        // the events live until every return below; on failure the previous
        // launch shape is kept
        struct Events {
            hipEvent_t e[2] = {nullptr, nullptr};
            ~Events()
            {
                for (hipEvent_t x : e)
                    if (x) (void)hipEventDestroy(x);
            }
        } ev;
        struct Restore {
            hermite_ctx *c;
            int ipt, nsplit, jsource, waves;
            bool keep = false;
            ~Restore()
            {
                if (keep) return;
                c->ipt = ipt;
                c->nsplit = nsplit;
                c->jsource = jsource;
                c->waves = waves;
            }
        } restore{ctx, ctx->ipt, ctx->nsplit, ctx->jsource, ctx->waves};
        HIP_TRY(ctx, hipEventCreate(&ev.e[0]), "event create");
        HIP_TRY(ctx, hipEventCreate(&ev.e[1]), "event create");
        std::vector<Timed> timed;
        for (const Cand &cd : shapes) {
            std::vector<int> cands;
            if (cd.src == 2) {
                // every pair once, when its partial sums fit; no j-split
                if (!pairs_fit(ctx, s->n)) continue;
                cands = {0};
            } else {
                const hermite::LaunchShape sh{cd.ipt, cd.waves,
                                              cd.src ? hermite::JSource::Scalar : hermite::JSource::Lds};
                const int base = hermite::auto_split(s->n, sh, false);
                cands = {base};
                for (int f : {2, 4}) {
                    if (base * f <= 64) cands.push_back(base * f);
                    if (base / f >= 1) cands.push_back(base / f);
                }
                std::sort(cands.begin(), cands.end());
                cands.erase(std::unique(cands.begin(), cands.end()), cands.end());
            }
            for (int ns : cands) {
                ctx->ipt = cd.ipt;
                ctx->waves = cd.waves;
                ctx->jsource = cd.src;
                ctx->nsplit = ns;
                st = hermite_force_derivs(ctx, s);   // warm-up
                if (st != HERMITE_OK) return st;
                HIP_TRY(ctx, hipEventRecord(ev.e[0], ctx->stream), "event record");
                for (int r = 0; r < 5; ++r) {
                    st = hermite_force_derivs(ctx, s);
                    if (st != HERMITE_OK) return st;
                }
                HIP_TRY(ctx, hipEventRecord(ev.e[1], ctx->stream), "event record");
                HIP_TRY(ctx, hipEventSynchronize(ev.e[1]), "event sync");
                float ms = 0.0f;
                HIP_TRY(ctx, hipEventElapsedTime(&ms, ev.e[0], ev.e[1]), "event time");
                const int64_t per_split = (int64_t)(ctx->p + 1) * 3 * s->n;
                const int64_t partials = cd.src == 2 ? hermite::pairs_partial_doubles(s->n, ctx->p)
                                         : ns > 1    ? (int64_t)ns * per_split
                                                     : 0;
                timed.push_back({cd, ns, ms, partials});
            }
        }
        restore.keep = true;
        // Fastest shape; among those within 2 % of it, the one that writes the
        // fewest partial sums (then the earliest in the list above).
        float best = 1e30f;
        for (const Timed &t : timed) best = std::min(best, t.ms);
        const Timed *pick = nullptr;
        for (const Timed &t : timed) {
            if (t.ms > 1.02f * best) continue;
            if (!pick || t.partials < pick->partials) pick = &t;
        }
        if (pick) {
            best_ipt = pick->c.ipt;
            best_waves = pick->c.waves;
            best_src = pick->c.src;
            best_split = pick->split;
            tune_cache().put(key, {best_ipt, best_split, best_src, best_waves});
        }
    }
    ctx->ipt = best_ipt;
    ctx->nsplit = best_split;
    ctx->jsource = best_src;
    ctx->waves = best_waves;
    if (i_per_thread) *i_per_thread = best_ipt;
    if (j_split) *j_split = best_split;
    if (j_source) *j_source = best_src;
    if (wg_waves) *wg_waves = best_waves;
    return HERMITE_OK;
}

// ---------------------------------------------------------------------------
// Batched form
// ---------------------------------------------------------------------------

hermite_status hermite_batch_create(const hermite_params *prm, int32_t n_sys, const int64_t *offsets,
                                    void *hip_stream, hermite_ctx **out)
{
    std::string msg;
    if (!out) return HERMITE_E_ARG;
    *out = nullptr;
    hermite_status st = check_params(prm, msg);
    if (st != HERMITE_OK) return st;
    if (prm->precision == HERMITE_SPLIT) return HERMITE_E_ARG;
    if (n_sys < 0 || (n_sys > 0 && !offsets)) return HERMITE_E_ARG;
    if (n_sys > 0 && offsets[0] != 0) return HERMITE_E_ARG;
    int32_t max_size = 0;
    for (int32_t i = 0; i < n_sys; ++i) {
        const int64_t sz = offsets[i + 1] - offsets[i];
        if (sz < 1 || sz > 64) return HERMITE_E_ARG;
        max_size = std::max<int32_t>(max_size, (int32_t)sz);
    }
    // First-fit-decreasing packing of systems into 64-lane bins.
    std::vector<int32_t> order(n_sys);
    for (int32_t i = 0; i < n_sys; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return offsets[a + 1] - offsets[a] > offsets[b + 1] - offsets[b];
    });
    std::vector<std::vector<int32_t>> bins;
    std::vector<int32_t> fill;
    for (int32_t s : order) {
        const int32_t sz = (int32_t)(offsets[s + 1] - offsets[s]);
        size_t b = 0;
        while (b < bins.size() && fill[b] + sz > 64) ++b;
        if (b == bins.size()) {
            bins.emplace_back();
            fill.push_back(0);
        }
        bins[b].push_back(s);
        fill[b] += sz;
    }
    std::vector<int32_t> bin_start(bins.size() + 1, 0), bin_sys;
    for (size_t b = 0; b < bins.size(); ++b) {
        bin_start[b + 1] = bin_start[b] + (int32_t)bins[b].size();
        for (int32_t s : bins[b]) bin_sys.push_back(s);
    }
    hermite_ctx *ctx = new hermite_ctx();
    ctx->prm = *prm;
    ctx->p = prm->order / 2 - 1;
    ctx->batch = true;
    ctx->n_sys = n_sys;
    ctx->n_bins = (int32_t)bins.size();
    ctx->max_size = max_size;
    ctx->offsets.assign(offsets, offsets + (n_sys + 1));
    ctx->n_max = n_sys > 0 ? offsets[n_sys] : 0;
    ctx->stream = (hipStream_t)hip_stream;
    auto alloc_copy = [&](void **dst, const void *src, size_t bytes) {
        if (bytes == 0) bytes = 8;
        if (hipMalloc(dst, bytes) != hipSuccess) return false;
        if (src && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return false;
        return true;
    };
    bool ok = alloc_copy((void **)&ctx->d_bin_start, bin_start.data(), bin_start.size() * sizeof(int32_t)) &&
              alloc_copy((void **)&ctx->d_bin_sys, bin_sys.empty() ? nullptr : bin_sys.data(),
                         bin_sys.size() * sizeof(int32_t)) &&
              alloc_copy((void **)&ctx->d_offsets, ctx->offsets.data(), ctx->offsets.size() * sizeof(int64_t)) &&
              alloc_copy((void **)&ctx->d_counter, nullptr, sizeof(int)) &&
              alloc_copy((void **)&ctx->d_iters, nullptr, (size_t)n_sys * sizeof(int32_t)) &&
              alloc_copy((void **)&ctx->flag, nullptr, sizeof(int)) &&
              hipHostMalloc((void **)&ctx->h_iters, (size_t)std::max(n_sys, 1) * sizeof(int32_t),
                            hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        return alloc_failed(ctx);
    }
    if (hipEventCreateWithFlags(&ctx->iters_copied, hipEventDisableTiming) != hipSuccess) {
        clear_hip_error();
        free_ctx(ctx);
        return HERMITE_E_HIP;
    }
    if (hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        clear_hip_error();
        free_ctx(ctx);
        return HERMITE_E_HIP;
    }
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
            clear_hip_error();
            cus = 256;
        }
        ctx->cus = cus;
    }
    ctx->bshape = default_batch_shape(ctx);
    *out = ctx;
    return HERMITE_OK;
}

static hermite::BatchPlan plan_of(hermite_ctx *ctx)
{
    hermite::BatchPlan pl{};
    pl.n_sys = ctx->n_sys;
    pl.n_bins = ctx->n_bins;
    pl.bin_start = ctx->d_bin_start;
    pl.bin_sys = ctx->d_bin_sys;
    pl.offsets = ctx->d_offsets;
    pl.counter = ctx->d_counter;
    return pl;
}

hermite_status hermite_batch_init(hermite_ctx *ctx, hermite_state *s)
{
    if (!ctx) return HERMITE_E_ARG;
    if (!ctx->batch) return fail(ctx, HERMITE_E_ARG, "hermite: not a batched context");
    hermite_status st = check_state(ctx, s, false, false);
    if (st != HERMITE_OK) return st;
    if (s->n != ctx->n_max) return fail(ctx, HERMITE_E_ARG, "hermite: state n differs from the batch total");
    HIP_TRY(ctx, hermite::launch_batch_init(plan_of(ctx), ctx->p, s->n, s->mass, s->pos, s->vel, s->deriv,
                                            ctx->prm.G, ctx->prm.eps2, ctx->stream),
            "batch init launch");
    if (ctx->prm.compensated && s->n > 0)
        HIP_TRY(ctx, hipMemsetAsync(s->comp, 0, (size_t)6 * s->n * sizeof(double), ctx->stream), "comp clear");
    s->initialized = 1;
    return HERMITE_OK;
}

static hermite_status batch_run_impl(hermite_ctx *ctx, hermite_state *s, const double *dt_sys, int32_t n_steps,
                                     int32_t n_iter, const int32_t *iters_host)
{
    if (!ctx) return HERMITE_E_ARG;
    if (!ctx->batch) return fail(ctx, HERMITE_E_ARG, "hermite: not a batched context");
    if (n_steps < 0) return fail(ctx, HERMITE_E_ARG, "hermite: n_steps must be >= 0");
    if (iters_host) {
        n_iter = 1;
        for (int32_t i = 0; i < ctx->n_sys; ++i) {
            if (iters_host[i] < 1 || iters_host[i] > 64)
                return fail(ctx, HERMITE_E_ARG, "hermite: every per-system n_iter must be in 1..64");
            n_iter = std::max(n_iter, iters_host[i]);
        }
    } else if (n_iter < 1) {
        return fail(ctx, HERMITE_E_ARG, "hermite: n_iter must be >= 1");
    }
    hermite_status st = check_state(ctx, s, true, false);
    if (st != HERMITE_OK) return st;
    if (s->n != ctx->n_max) return fail(ctx, HERMITE_E_ARG, "hermite: state n differs from the batch total");
    if (ctx->n_sys > 0 && !dt_sys) return fail(ctx, HERMITE_E_ARG, "hermite: dt_sys is NULL");
    if (n_steps == 0 || ctx->n_sys == 0) return HERMITE_OK;
    if (iters_host) {
        // The counts are read here, into the pinned staging buffer, once the
        // previous call's copy out of it has run; the caller's array is free
        // again when this call returns.
        HIP_TRY(ctx, hipEventSynchronize(ctx->iters_copied), "per-system n_iter staging wait");
        std::memcpy(ctx->h_iters, iters_host, (size_t)ctx->n_sys * sizeof(int32_t));
        HIP_TRY(ctx, hipMemcpyAsync(ctx->d_iters, ctx->h_iters, (size_t)ctx->n_sys * sizeof(int32_t),
                                    hipMemcpyHostToDevice, ctx->stream),
                "per-system n_iter copy");
        HIP_TRY(ctx, hipEventRecord(ctx->iters_copied, ctx->stream), "per-system n_iter event");
    }
    hermite::BatchShape sh = ctx->bshape;
    sh.workgroups = std::max(1, std::min<int>(ctx->n_bins, sh.workgroups));
    const bool per_system = iters_host != nullptr;
    hermite_ctx::Key key{s->mass, dt_sys, s->pos, s->vel, s->deriv, comp_of(ctx, s), n_steps,
                         per_system ? 0 : n_iter, sh, per_system};
    if (!ctx->graph_exec || !(key == ctx->key)) {
        if (ctx->graph_exec) { (void)hipGraphExecDestroy(ctx->graph_exec); ctx->graph_exec = nullptr; }
        if (ctx->graph) { (void)hipGraphDestroy(ctx->graph); ctx->graph = nullptr; }
        hipStream_t cs = ctx->capture_stream;
        HIP_TRY(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "graph capture begin");
        hipError_t e1 = hermite::launch_reset_counter(ctx->d_counter, cs);
        hipError_t e2 = hermite::launch_batch_run(plan_of(ctx), ctx->p, ctx->prm.precision == HERMITE_MIXED,
                                                  ctx->prm.corrector, s->n, s->mass, s->pos, s->vel, s->deriv,
                                                  dt_sys, n_steps, n_iter, per_system ? ctx->d_iters : nullptr,
                                                  ctx->prm.G, ctx->prm.eps2, comp_of(ctx, s), sh, cs);
        hipGraph_t g = nullptr;
        hipError_t e3 = hipStreamEndCapture(cs, &g);
        if (e1 != hipSuccess) return hip_fail(ctx, e1, "graph capture (counter reset)");
        if (e2 != hipSuccess) return hip_fail(ctx, e2, "graph capture (batch kernel)");
        if (e3 != hipSuccess) return hip_fail(ctx, e3, "graph capture end");
        ctx->graph = g;
        HIP_TRY(ctx, hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0), "graph instantiate");
        ctx->key = key;
    }
    HIP_TRY(ctx, hipGraphLaunch(ctx->graph_exec, ctx->stream), "graph launch");
    s->t += n_steps;
    if (!ctx->prm.check_finite) return HERMITE_OK;
    const double *arrs[3] = {s->pos, s->vel, s->deriv};
    const int64_t cnt[3] = {3 * s->n, 3 * s->n, (int64_t)2 * ctx->p * 3 * s->n};
    return check_finite(ctx, arrs, cnt, 3);
}

hermite_status hermite_batch_set_launch(hermite_ctx *ctx, int32_t workgroups, int32_t waves, int32_t ring_min)
{
    if (!ctx) return HERMITE_E_ARG;
    if (!ctx->batch) return fail(ctx, HERMITE_E_ARG, "hermite: not a batched context");
    if (workgroups < 0) return fail(ctx, HERMITE_E_ARG, "hermite: workgroups must be >= 0");
    if (waves != 1 && waves != 2 && waves != 4) return fail(ctx, HERMITE_E_ARG, "hermite: waves must be 1, 2 or 4");
    if (ring_min < 2 || ring_min > 65) return fail(ctx, HERMITE_E_ARG, "hermite: ring_min must be in 2..65");
    hermite::BatchShape sh{workgroups, waves, ring_min};
    if (workgroups == 0) sh.workgroups = batch_resident(ctx, sh);
    ctx->bshape = sh;
    ctx->bshape_set = true;
    return HERMITE_OK;
}

hermite_status hermite_batch_get_launch(hermite_ctx *ctx, int32_t *workgroups, int32_t *waves, int32_t *ring_min)
{
    if (!ctx) return HERMITE_E_ARG;
    if (!ctx->batch) return fail(ctx, HERMITE_E_ARG, "hermite: not a batched context");
    if (workgroups) *workgroups = std::max(1, std::min(ctx->n_bins, ctx->bshape.workgroups));
    if (waves) *waves = ctx->bshape.waves;
    if (ring_min) *ring_min = ctx->bshape.ring_min;
    return HERMITE_OK;
}

hermite_status hermite_batch_autotune(hermite_ctx *ctx, hermite_state *s, const double *dt_sys, int32_t n_steps,
                                      int32_t n_iter, int32_t *workgroups, int32_t *waves, int32_t *ring_min,
                                      int32_t *from_cache)
{
    if (!ctx) return HERMITE_E_ARG;
    if (!ctx->batch) return fail(ctx, HERMITE_E_ARG, "hermite: not a batched context");
    if (n_steps < 1) return fail(ctx, HERMITE_E_ARG, "hermite: n_steps must be >= 1");
    if (n_iter < 1 || n_iter > 64) return fail(ctx, HERMITE_E_ARG, "hermite: n_iter must be in 1..64");
    hermite_status st = check_state(ctx, s, true, false);
    if (st != HERMITE_OK) return st;
    if (s->n != ctx->n_max) return fail(ctx, HERMITE_E_ARG, "hermite: state n differs from the batch total");
    if (ctx->n_sys > 0 && !dt_sys) return fail(ctx, HERMITE_E_ARG, "hermite: dt_sys is NULL");
    auto report = [&](bool cached) {
        (void)hermite_batch_get_launch(ctx, workgroups, waves, ring_min);
        if (from_cache) *from_cache = cached ? 1 : 0;
        return HERMITE_OK;
    };
    if (ctx->n_sys == 0) return report(false);
    // cache key: order, precision, compensation, iterations, the histogram of
    // system sizes (FNV-1a over the 64 counts), the bin count and the device
    uint64_t hsh = 1469598103934665603ull;
    {
        int64_t hist[65] = {};
        for (int32_t i = 0; i < ctx->n_sys; ++i) ++hist[ctx->offsets[i + 1] - ctx->offsets[i]];
        for (int k = 1; k <= 64; ++k)
            for (int b = 0; b < 8; ++b) {
                hsh ^= (uint64_t)((hist[k] >> (8 * b)) & 0xff);
                hsh *= 1099511628211ull;
            }
    }
    char key[512];
    std::snprintf(key, sizeof key, "batch|p=%d|prec=%d|comp=%d|n_iter=%d|sizes=%016llx|bins=%d|dev=%s", ctx->p,
                  ctx->prm.precision, ctx->prm.compensated, n_iter, (unsigned long long)hsh, ctx->n_bins,
                  device_tag().c_str());
    std::vector<int> cached;
    if (tune_cache().get(key, cached) && cached.size() == 3) {
        const hermite::BatchShape sh{cached[0], cached[1], cached[2]};
        if (hermite::batch_shape_ok(sh)) {
            ctx->bshape = sh;
            ctx->bshape_set = true;
            return report(true);
        }
    }
    // Time every candidate on a copy of the state (the caller's is left
    // alone), each from the same starting point.
    const int64_t n3 = 3 * s->n;
    const size_t sbytes = (size_t)(2 + 2 * ctx->p) * n3 * sizeof(double);   // x, v, a^(0..2p-1)
    const size_t cbytes = ctx->prm.compensated ? (size_t)2 * n3 * sizeof(double) : 0;
    struct Scratch {
        double *buf = nullptr;
        hipEvent_t e[2] = {nullptr, nullptr};
        ~Scratch()
        {
            if (buf) (void)hipFree(buf);
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } sc;
    if (hipMalloc((void **)&sc.buf, 2 * (sbytes + cbytes)) != hipSuccess) {
        clear_hip_error();
        return fail(ctx, HERMITE_E_ALLOC, "hermite: batched autotune could not allocate its state copy");
    }
    HIP_TRY(ctx, hipEventCreate(&sc.e[0]), "event create");
    HIP_TRY(ctx, hipEventCreate(&sc.e[1]), "event create");
    double *orig = sc.buf;                                   // pristine copy: x, v, deriv, comp
    double *work = sc.buf + (sbytes + cbytes) / sizeof(double);
    auto copy_state = [&](double *dst, const double *x, const double *v, const double *d, const double *c) {
        hipError_t e = hipMemcpyAsync(dst, x, n3 * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dst + n3, v, n3 * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dst + 2 * n3, d, (size_t)2 * ctx->p * n3 * sizeof(double), hipMemcpyDeviceToDevice,
                               ctx->stream);
        if (e == hipSuccess && cbytes)
            e = hipMemcpyAsync(dst + sbytes / sizeof(double), c, cbytes, hipMemcpyDeviceToDevice, ctx->stream);
        return e;
    };
    HIP_TRY(ctx, copy_state(orig, s->pos, s->vel, s->deriv, comp_of(ctx, s)), "autotune state copy");
    double *wx = work, *wv = work + n3, *wd = work + 2 * n3, *wc = cbytes ? work + sbytes / sizeof(double) : nullptr;
    std::vector<hermite::BatchShape> cands;
    for (int wv_ : {1, 2, 4})
        for (int rm : {57, 65}) {
            hermite::BatchShape sh{0, wv_, rm};
            const int res = batch_resident(ctx, sh);
            const int per_cu = std::max(1, res / std::max(1, ctx->cus));
            // from half the resident workgroups to all of them, per CU
            for (int k = std::max(1, per_cu / 2); k <= per_cu; ++k) {
                sh.workgroups = std::min(ctx->n_bins, k * ctx->cus);
                cands.push_back(sh);
            }
        }
    hermite::BatchShape best = ctx->bshape;
    float best_ms = 1e30f;
    for (const hermite::BatchShape &sh : cands) {
        float ms = 0.0f;
        for (int rep = 0; rep < 2; ++rep) {   // a warm-up run, then the timed one
            HIP_TRY(ctx, copy_state(work, orig, orig + n3, orig + 2 * n3, cbytes ? orig + sbytes / sizeof(double) : nullptr),
                    "autotune state copy");
            HIP_TRY(ctx, hipEventRecord(sc.e[0], ctx->stream), "event record");
            HIP_TRY(ctx, hermite::launch_reset_counter(ctx->d_counter, ctx->stream), "autotune counter reset");
            HIP_TRY(ctx, hermite::launch_batch_run(plan_of(ctx), ctx->p, ctx->prm.precision == HERMITE_MIXED,
                                                   ctx->prm.corrector, s->n, s->mass, wx, wv, wd, dt_sys, n_steps,
                                                   n_iter, nullptr, ctx->prm.G, ctx->prm.eps2, wc, sh, ctx->stream),
                    "autotune batch launch");
            HIP_TRY(ctx, hipEventRecord(sc.e[1], ctx->stream), "event record");
            HIP_TRY(ctx, hipEventSynchronize(sc.e[1]), "event sync");
            HIP_TRY(ctx, hipEventElapsedTime(&ms, sc.e[0], sc.e[1]), "event time");
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = sh;
        }
    }
    ctx->bshape = best;
    ctx->bshape_set = true;
    tune_cache().put(key, {best.workgroups, best.waves, best.ring_min});
    return report(false);
}

void hermite_tune_cache_clear(void) { tune_cache().clear(); }

static_assert(sizeof(hermite_vstep_cfg) == sizeof(hermite::EnsembleCfg), "cfg layout");
static_assert(sizeof(hermite_vstep_result) == sizeof(hermite::EnsembleStatus), "result layout");

hermite_status hermite_ensemble_create(const hermite_params *prm, int32_t n_sys, const int64_t *offsets,
                                       void *hip_stream, hermite_ctx **out)
{
    std::string msg;
    if (!out) return HERMITE_E_ARG;
    *out = nullptr;
    hermite_status st = check_params(prm, msg);
    if (st != HERMITE_OK) return st;
    if (prm->precision != HERMITE_FP64 || prm->compensated) return HERMITE_E_ARG;
    if (n_sys < 0 || (n_sys > 0 && !offsets)) return HERMITE_E_ARG;
    if (n_sys > 0 && offsets[0] != 0) return HERMITE_E_ARG;
    for (int32_t i = 0; i < n_sys; ++i) {
        const int64_t sz = offsets[i + 1] - offsets[i];
        if (sz < 2 || sz > 128) return HERMITE_E_ARG;
    }
    hermite_ctx *ctx = new hermite_ctx();
    ctx->prm = *prm;
    ctx->p = prm->order / 2 - 1;
    ctx->ensemble = true;
    ctx->n_sys = n_sys;
    ctx->offsets.assign(offsets, offsets + (n_sys + 1));
    ctx->n_max = n_sys > 0 ? offsets[n_sys] : 0;
    ctx->stream = (hipStream_t)hip_stream;
    const size_t ns = (size_t)std::max(n_sys, 1);
    bool ok = hipMalloc((void **)&ctx->d_offsets, (ns + 1) * sizeof(int64_t)) == hipSuccess &&
              hipMalloc((void **)&ctx->d_cfg, ns * sizeof(hermite::EnsembleCfg)) == hipSuccess &&
              hipMalloc((void **)&ctx->d_status, ns * sizeof(hermite::EnsembleStatus)) == hipSuccess &&
              hipMalloc((void **)&ctx->flag, sizeof(int)) == hipSuccess;
    if (ok && n_sys > 0)
        ok = hipMemcpy(ctx->d_offsets, offsets, (size_t)(n_sys + 1) * sizeof(int64_t), hipMemcpyHostToDevice) ==
             hipSuccess;
    if (!ok) {
        return alloc_failed(ctx);
    }
    *out = ctx;
    return HERMITE_OK;
}

hermite_status hermite_ensemble_init(hermite_ctx *ctx, hermite_state *s)
{
    if (!ctx) return HERMITE_E_ARG;
    if (!ctx->ensemble) return fail(ctx, HERMITE_E_ARG, "hermite: not an ensemble context");
    hermite_status st = check_state(ctx, s, false, false);
    if (st != HERMITE_OK) return st;
    if (s->n != ctx->n_max) return fail(ctx, HERMITE_E_ARG, "hermite: state n differs from the ensemble total");
    if (ctx->n_sys == 0) {
        s->initialized = 1;
        return HERMITE_OK;
    }
    HIP_TRY(ctx, hermite::launch_ensemble_init(ctx->d_offsets, ctx->n_sys, ctx->p, s->n, s->mass, s->pos, s->vel,
                                               s->deriv, ctx->prm.G, ctx->prm.eps2, ctx->stream),
            "ensemble init launch");
    HIP_TRY(ctx, hipMemsetAsync(ctx->d_status, 0, (size_t)ctx->n_sys * sizeof(hermite::EnsembleStatus), ctx->stream),
            "ensemble status clear");
    s->initialized = 1;
    return HERMITE_OK;
}

hermite_status hermite_ensemble_run(hermite_ctx *ctx, hermite_state *s, const hermite_vstep_cfg *cfg,
                                    int64_t max_steps, int32_t rec_cap, double *rec, hermite_vstep_result *res)
{
    if (!ctx) return HERMITE_E_ARG;
    if (!ctx->ensemble) return fail(ctx, HERMITE_E_ARG, "hermite: not an ensemble context");
    hermite_status st = check_state(ctx, s, true, false);
    if (st != HERMITE_OK) return st;
    if (s->n != ctx->n_max) return fail(ctx, HERMITE_E_ARG, "hermite: state n differs from the ensemble total");
    if (max_steps < 0) return fail(ctx, HERMITE_E_ARG, "hermite: max_steps must be >= 0");
    if (rec_cap < 0 || (rec_cap > 0 && !rec)) return fail(ctx, HERMITE_E_ARG, "hermite: bad record buffer");
    if (ctx->n_sys > 0 && (!cfg || !res)) return fail(ctx, HERMITE_E_ARG, "hermite: cfg and res are required");
    for (int32_t i = 0; i < ctx->n_sys; ++i) {
        const hermite_vstep_cfg &c = cfg[i];
        if (!std::isfinite(c.eta) || !(c.eta > 0.0) || !std::isfinite(c.t_end) || std::isnan(c.rec_from) ||
            c.n_iter < 1 || c.n_iter > 64)
            return fail(ctx, HERMITE_E_ARG,
                        "hermite: each system needs eta finite and > 0, t_end finite, rec_from not NaN, "
                        "n_iter in 1..64");
    }
    if (ctx->n_sys == 0) return HERMITE_OK;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->d_cfg, cfg, (size_t)ctx->n_sys * sizeof(hermite::EnsembleCfg),
                                hipMemcpyHostToDevice, ctx->stream),
            "ensemble cfg copy");
    hermite::EnsembleArgs a{};
    a.n_sys = ctx->n_sys;
    a.n = s->n;
    a.offsets = ctx->d_offsets;
    a.mass = s->mass;
    a.pos = s->pos;
    a.vel = s->vel;
    a.deriv = s->deriv;
    a.G = ctx->prm.G;
    a.eps2 = ctx->prm.eps2;
    a.cfg = ctx->d_cfg;
    a.status = ctx->d_status;
    a.rec = rec;
    a.rec_cap = rec_cap;
    a.max_steps = max_steps;
    if (max_steps > 0)
        HIP_TRY(ctx, hermite::launch_ensemble_run(a, ctx->p, ctx->prm.corrector, ctx->stream), "ensemble run launch");
    HIP_TRY(ctx, hipMemcpyAsync(res, ctx->d_status, (size_t)ctx->n_sys * sizeof(hermite::EnsembleStatus),
                                hipMemcpyDeviceToHost, ctx->stream),
            "ensemble status copy");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "ensemble sync");
    for (int32_t i = 0; i < ctx->n_sys; ++i)
        if (res[i].failed)
            return fail(ctx, HERMITE_E_NONFINITE,
                        "hermite: the step criterion became undefined in a system (see its result's failed flag)");
    return HERMITE_OK;
}

hermite_status hermite_batch_run(hermite_ctx *ctx, hermite_state *s, const double *dt_sys, int32_t n_steps,
                                 int32_t n_iter)
{
    return batch_run_impl(ctx, s, dt_sys, n_steps, n_iter, nullptr);
}

hermite_status hermite_batch_run_iters(hermite_ctx *ctx, hermite_state *s, const double *dt_sys, int32_t n_steps,
                                       const int32_t *n_iter_sys)
{
    if (ctx && ctx->n_sys > 0 && !n_iter_sys) return fail(ctx, HERMITE_E_ARG, "hermite: n_iter_sys is NULL");
    return batch_run_impl(ctx, s, dt_sys, n_steps, 0, n_iter_sys ? n_iter_sys : nullptr);
}

}  // extern "C"
