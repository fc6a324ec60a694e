/*
 * hermite.h -- C ABI of the MI355X (gfx950) modified Hermite N-body hot path.
 *
 * Method: A. J. Dittmann, "Modified Hermite Integrators of Arbitrary Order"
 * (MNRAS 2020, arXiv:2006.02501).  An order-2(p+1) scheme (p = 1, 2, 3 for
 * 4th, 6th, 8th order; Sec. 2, after Eq. 8) evaluates the softened pair
 * acceleration a_ij = G m_j r_ij (r_ij^2 + eps^2)^(-3/2) (Sec. 3, opening
 * paragraph) and its first p time derivatives by direct O(N^2) summation,
 * once per predict-evaluate-correct iteration of a P(EC)^n step (Sec. 2.1,
 * end); between evaluations it runs a Taylor predictor and the modified
 * corrector of Eq. 22-24 (velocity first, then position; Eq. 6-8).
 *
 * Conventions shared by every call
 * --------------------------------
 * - All particle arrays are DEVICE pointers to FP64 data owned by the caller
 *   (e.g. torch tensors), laid out structure-of-arrays: a "[3][n] block" is
 *   x-components of all n particles, then y, then z.  "[k][3][n]" is k such
 *   blocks back to back.  The library never frees or reallocates them.
 * - The library owns only its workspace (split partial sums, batched-plan
 *   tables, the captured graph), allocated in *_create and freed in
 *   hermite_destroy.
 * - Every call is asynchronous on the HIP stream given to *_create (NULL =
 *   the null stream).  Only hermite_last_error and the optional finite-value
 *   check synchronise.
 * - Arguments are validated on the host before any HIP call; a bad argument
 *   returns an error code and enqueues nothing.  Nothing is thrown across the
 *   ABI.  After an error, hermite_last_error(ctx) gives a message.
 * - One context is used by one host thread at a time.
 * - Results are bitwise reproducible for a given context configuration and
 *   n: the sums use a fixed order and no atomics.
 * - Negative dt integrates backwards with the same formulas.
 */
#ifndef HERMITE_H
#define HERMITE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hermite_ctx hermite_ctx;

typedef enum {
    HERMITE_OK = 0,
    HERMITE_E_ARG = -1,        /* bad pointer, size, dt, n_iter, eps2, ...          */
    HERMITE_E_ORDER = -2,      /* order not in {4, 6, 8}                           */
    HERMITE_E_ALLOC = -3,      /* device allocation failed / workspace too small   */
    HERMITE_E_HIP = -4,        /* a HIP runtime call failed (message kept)         */
    HERMITE_E_NONFINITE = -5,  /* finite check enabled and a result is inf / NaN   */
    HERMITE_E_STATE = -6       /* called before hermite_init on this state         */
} hermite_status;

typedef enum {
    HERMITE_FP64 = 0,   /* every operation in FP64                                   */
    HERMITE_MIXED = 1,  /* FP64 state and pairwise differences; the r^-3 pair term
                           and its derivative chain in FP32, summed in FP32 over
                           32 j at a time and in FP64 across those sums          */
    HERMITE_SPLIT = 2   /* the paper's own suggestion (Sec. 4: lower precision for
                           the higher-order terms on accelerators): a and adot
                           exactly as HERMITE_FP64 computes them (bitwise, for a
                           given launch shape), a^(2) and a^(3) in FP32 as in
                           HERMITE_MIXED.  At 4th order it is HERMITE_FP64.
                           Not available in the batched form (E_ARG there).      */
} hermite_precision;

typedef enum {
    HERMITE_CORR_MODIFIED = 0,  /* beta_opt of Eq. 21: Eq. 22 / 23 / 24 (default)     */
    HERMITE_CORR_BETA1 = 1,     /* beta = 1: the position formula exact one order
                                   higher (the standard time-symmetric corrector at
                                   4th order, Sec. 3.1)                               */
    HERMITE_CORR_SHIFTED = 2    /* beta = 2 - beta_opt: drops the F_{2p+2} term's
                                   endpoint derivative (the unmodified 6th/8th-order
                                   correctors the paper compares against)            */
} hermite_corrector;

typedef struct {
    int32_t order;         /* 4, 6 or 8 (= 2(p+1))                                  */
    int32_t precision;     /* hermite_precision                                     */
    int32_t corrector;     /* hermite_corrector                                     */
    int32_t check_finite;  /* nonzero: hermite_step / hermite_batch_run check every
                              output for inf / NaN (synchronises; E_NONFINITE)     */
    double G;              /* gravitational constant                                */
    double eps2;           /* softening eps^2 >= 0 (Sec. 3: eps = 1e-8 or 1e-6)     */
    int32_t compensated;   /* nonzero: x, v and t take each step's increments by
                              compensated (Kahan) summation, the option Sec. 3.2
                              uses for its 8th-order runs; the state then carries
                              the compensation terms (comp, t_comp).  The
                              batched form compensates x and v (its t is a step
                              count); the ensemble form does not offer it (E_ARG). */
    int32_t reserved;      /* set to 0                                              */
} hermite_params;

/*
 * Particle state, p = order/2 - 1.  All pointers are device pointers, FP64,
 * caller-owned, SoA as described above.
 *   mass   [n]
 *   pos    [3][n]        x at time t
 *   vel    [3][n]        v at time t
 *   deriv  [2p][3][n]    a^(0..2p-1) at time t (a, adot, a^(2), ..., written by
 *                        hermite_init, advanced by the last correction of a step)
 *   pred   [p+1][3][n]   the path of the current iterate: x, v and, for p >= 2,
 *                        a (and adot for p = 3) -- what the evaluation reads
 *   eval   [p+1][3][n]   a^(0..p) from the latest evaluation
 * t is a host scalar advanced by the last correction of each step.
 * initialized is set to 1 by hermite_init (a caller restoring a saved state
 * sets it itself: (t, mass, pos, vel, deriv) is the complete state, plus
 * (comp, t_comp) with compensated summation).
 */
typedef struct {
    int64_t n;
    const double *mass;
    double *pos;
    double *vel;
    double *deriv;
    double *pred;
    double *eval;
    double t;
    int32_t initialized;
    int32_t reserved;
    double *comp;          /* [2][3][n] compensation terms of x and v (used only with
                              params.compensated; hermite_init zeroes them)       */
    double t_comp;         /* compensation term of t (same)                         */
} hermite_state;

/* Create a context for states of up to n_max particles (0 <= n_max <= 2^40).
 * hip_stream is a hipStream_t (NULL = null stream).  Validates *prm:
 * order -> E_ORDER; precision/corrector out of range, G not finite,
 * eps2 < 0 or not finite, n_max outside [0, 2^40], out NULL -> E_ARG.
 * Allocates the split-sum workspace for n_max (E_ALLOC on failure). */
hermite_status hermite_create(const hermite_params *prm, int64_t n_max, void *hip_stream,
                              hermite_ctx **out);

/* Free the workspace and the context (NULL is accepted). */
hermite_status hermite_destroy(hermite_ctx *ctx);

/* Change the stream later calls are enqueued on. */
hermite_status hermite_set_stream(hermite_ctx *ctx, void *hip_stream);

/* Explicit initial derivatives (Sec. 3, second paragraph): a^(0..2p-1) at t
 * from pos and vel by passes of the generic-order pair derivative
 * (a, adot from x, v; then a^(2), a^(3); then, at 8th order, a^(4), a^(5)),
 * always in FP64.  Writes s->deriv (uses s->eval and s->pred as scratch),
 * zeroes s->comp and s->t_comp with compensated summation, sets
 * s->initialized.  E_ARG on NULL pointers (comp too, when compensated) or
 * n > n_max. */
hermite_status hermite_init(hermite_ctx *ctx, hermite_state *s);

/* Taylor predictor (Sec. 3, second paragraph) with every stored derivative:
 * x to dt^(2p+1), v to dt^(2p), a to dt^(2p-1), adot to dt^(2p-2).
 * Writes s->pred.  E_ARG if dt is 0 or not finite; E_STATE before init. */
hermite_status hermite_predict(hermite_ctx *ctx, hermite_state *s, double dt);

/* One evaluation (the O(N^2) hot loop): for every i,
 *   a^(k)_i = sum_{j != i} d^k/dt^k [ G m_j r_ij (r_ij^2 + eps^2)^(-3/2) ],
 * k = 0..p, along the path s->pred (x, v, a, adot of every particle).
 * Self terms are excluded by index.  Writes s->eval. */
hermite_status hermite_force_derivs(hermite_ctx *ctx, hermite_state *s);

/* The same evaluation for the i-particles [i0, i0 + ni) only, each against
 * every j != i: the share of one GPU when the particles are divided among
 * GPUs by i (all the paths gathered on every GPU).  Writes s->eval at those
 * positions ([p+1][3][n] layout) and leaves the others alone.  It takes the
 * context's launch shape when that is one-sided (j_source 0 or 1); with
 * j_source 2 (every pair once, which has no one-sided form) the LDS source
 * with two i-particles per lane (FP64, split) or the scalar source with one
 * (mixed).  E_ARG for a range outside [0, n). */
hermite_status hermite_force_derivs_range(hermite_ctx *ctx, hermite_state *s, int64_t i0, int64_t ni);

/* Modified corrector (Eq. 6-8; Eq. 22-24 for the default corrector) from
 * the start-of-step state (pos, vel, deriv[0..p]) and s->eval:
 *   v1 = v0 + sum_{k=0..p}   cv_k (a1^(k) +- a0^(k)) dt^(k+1)
 *   x1 = x0 + sum_{k=0..p+1} cx_k (q1^(k) +- q0^(k)) dt^(k+1),  q = (v, a, adot, ...)
 * (+ for even k, - for odd k).  last_iter == 0: writes the next iterate into
 * s->pred (x1, v1 and the evaluated a, adot as the relative-acceleration path).
 * last_iter != 0: overwrites pos, vel with x1, v1, sets deriv[0..p] = eval
 * and deriv[p+1..2p-1] to the Hermite interpolant's derivatives at the end of
 * the step, and advances s->t by dt. */
hermite_status hermite_correct(hermite_ctx *ctx, hermite_state *s, double dt, int32_t last_iter);

/* One P(EC)^n step: predict, then n_iter times (force_derivs, correct),
 * the last correction with last_iter = 1.  E_ARG if n_iter < 1. */
hermite_status hermite_step(hermite_ctx *ctx, hermite_state *s, double dt, int32_t n_iter);

/*
 * Variable, time-symmetric step (Sec. 3.3, Eq. 25).  The criterion is
 *   H(x) = eta min_{i != j} ((r_ij^2 + eps^2)^(3/2) / (G (m_i + m_j)))^(1/2),
 * the shortest two-body Kepler time scale over all pairs, times eta.
 *
 * hermite_step_criterion: H at s->pos into the host double *h (synchronises).
 * E_ARG if n < 2, eta is not finite and > 0, or h is NULL; E_NONFINITE if H
 * is not finite and positive (no pair with G (m_i + m_j) > 0, coincident
 * bodies without softening, non-finite positions).
 *
 * hermite_step_symmetric: one P(EC)^n step whose length is chosen implicitly
 * as the iteration proceeds, dt = direction * (H_- + H_+) / 2 with H at the
 * start and at the end of the step.  H_- = H(x0); the Taylor prediction for
 * dt = direction * H_- gives a first end point, H_+ there gives dt_1, and the
 * prediction is redone for dt_1.  Iteration k evaluates at its path, which
 * lies at t0 + dt_k, and corrects with that same dt_k (the corrector's end
 * values belong to the end of the step it makes, Eq. 4-8).  Before the next
 * iteration, H_+ at this evaluation point gives dt_(k+1) and the iterate
 * (x1, v1, a1^(0..p)) is moved to t0 + dt_(k+1) along its Taylor series to
 * form the next path.  Converged iterations give a step that is the same
 * taken forwards or backwards.  The step taken is the last correction's dt,
 * which stays on the
 * device between launches; at the end it is copied back (synchronises),
 * added to s->t and stored in *dt_taken (host, may be NULL).
 * direction is +1 (forwards) or -1 (backwards).  E_ARG for n < 2, n_iter < 1,
 * eta not finite and > 0, other directions; E_STATE before init;
 * E_NONFINITE when H is undefined at any point of the step, in which case
 * pos, vel, deriv and t are left unchanged (pred and eval are scratch).
 */
hermite_status hermite_step_criterion(hermite_ctx *ctx, const hermite_state *s, double eta, double *h);
hermite_status hermite_step_symmetric(hermite_ctx *ctx, hermite_state *s, double eta, int32_t n_iter,
                                      double direction, double *dt_taken);

/* Energy diagnostic (Sec. 3.1): phi[i] = -sum_{j != i} G m_j (r_ij^2+eps^2)^(-1/2)
 * at s->pos, FP64, written to the device array phi[n]. */
hermite_status hermite_potential(hermite_ctx *ctx, const hermite_state *s, double *phi);

/*
 * Batched form: n_sys independent systems concatenated in one state
 * (particles offsets[s] .. offsets[s+1]-1 belong to system s; offsets is a
 * HOST array of n_sys+1 nondecreasing values starting at 0, each system of
 * 1..64 particles).  Pair sums run only inside a system.  precision
 * HERMITE_SPLIT is not offered (E_ARG).  With params.compensated the state's
 * comp array is required and hermite_batch_init zeroes it.  All steps of all
 * systems run in one persistent kernel launch (launch shape: see
 * hermite_batch_set_launch), replayed from a captured HIP graph; systems are
 * packed into 64-slot bins and handed out longest first from a device work
 * counter.  An evaluation takes every pair of a system once, for both of its
 * bodies (sums in another order than the single-system path, the same to
 * rounding).
 */
hermite_status hermite_batch_create(const hermite_params *prm, int32_t n_sys, const int64_t *offsets,
                                    void *hip_stream, hermite_ctx **out);

/* Explicit initial derivatives of every system (FP64), as hermite_init. */
hermite_status hermite_batch_init(hermite_ctx *ctx, hermite_state *s);

/* n_steps P(EC)^n steps of every system; dt_sys is a DEVICE array [n_sys] of
 * per-system steps.  Updates pos, vel, deriv in place (pred and eval are not
 * used).  s->t is advanced by n_steps (per-system times are n_steps*dt_sys). */
hermite_status hermite_batch_run(hermite_ctx *ctx, hermite_state *s, const double *dt_sys,
                                 int32_t n_steps, int32_t n_iter);

/* The same with an iteration count per system: n_iter_sys is a HOST array
 * [n_sys] of values in 1..64 (E_ARG otherwise).  It is read during the call
 * (staged through a pinned buffer of the context), so the caller may change
 * or free it as soon as the call returns.  A bin of systems iterates as often
 * as its largest count; each
 * system corrects only its own n times and keeps that iterate (the paper's
 * n-sweep, Sec. 3.1, runs every n side by side this way). */
hermite_status hermite_batch_run_iters(hermite_ctx *ctx, hermite_state *s, const double *dt_sys,
                                       int32_t n_steps, const int32_t *n_iter_sys);

/*
 * Launch shape of the batched run.  All waves of a workgroup work on one bin
 * of systems at a time; the workgroups are persistent and take bins from a
 * device counter.
 *   workgroups  persistent workgroups (0: as many as the GPU holds at once;
 *               at most the bin count are launched)
 *   waves       wave64 per workgroup, 1, 2 or 4: the waves split each
 *               evaluation's sweep steps between them and the per-body work
 *               (predictor, corrector) by coordinate component; their sums are
 *               added through LDS in wave order
 *   ring_min    bins whose largest system has at least ring_min bodies sweep
 *               the whole wave as one ring, the j-side sums of a pair moving
 *               between lanes by DPP; the others sweep each system as a ring
 *               of its own, the sums moving by lane permutes (through LDS with
 *               two or more waves) (2..65; 65: never)
 * Results are bitwise the same for every workgroup count (each bin is
 * computed by one workgroup in a fixed order); waves and ring_min change the
 * order of the sums, hence the rounding.  E_ARG for values outside these
 * sets or a context that is not batched.  hermite_batch_get_launch reports
 * the shape in use (the creation default: 2 waves, 1 when no system has
 * more than 16 bodies, 4 when every bin fits on the GPU at once with 4 waves
 * each; ring_min 57; every resident workgroup).
 *
 * hermite_batch_autotune times every supported shape (waves 1, 2, 4;
 * ring_min 57 or none; from half to all of the resident workgroups) for
 * n_steps steps of n_iter iterations on a device copy of the given state (the
 * state itself is not changed; the copy is allocated and freed inside the
 * call, which synchronises), keeps the fastest and returns it through the
 * non-NULL out pointers.  The pick is cached for the process (and, when the
 * environment variable HERMITE_TUNE_CACHE names a file, in that file), keyed
 * by order, precision, compensation, n_iter, the histogram of system sizes,
 * the bin count and the device's architecture and CU count; a cached pick is
 * returned without timing (*from_cache = 1).  hermite_autotune caches its
 * picks the same way (keyed by order, precision, a quarter-octave bucket of n
 * and the device).  hermite_tune_cache_clear forgets the cached picks of the
 * process (not the file's).
 */
hermite_status hermite_batch_set_launch(hermite_ctx *ctx, int32_t workgroups, int32_t waves, int32_t ring_min);
hermite_status hermite_batch_get_launch(hermite_ctx *ctx, int32_t *workgroups, int32_t *waves, int32_t *ring_min);
hermite_status hermite_batch_autotune(hermite_ctx *ctx, hermite_state *s, const double *dt_sys, int32_t n_steps,
                                      int32_t n_iter, int32_t *workgroups, int32_t *waves, int32_t *ring_min,
                                      int32_t *from_cache);
void hermite_tune_cache_clear(void);

/*
 * Ensemble form (Sec. 3.3 N-body test, Table 1): n_sys independent systems of
 * 2..128 bodies (offsets as for the batched form, HOST array), FP64, each
 * integrated by one workgroup with the variable time-symmetric step (the
 * criterion and step rule of hermite_step_symmetric, forwards) for many
 * steps inside one launch.  Every system keeps its own time on the device,
 * starting at 0 at hermite_ensemble_init.
 *
 * hermite_ensemble_create: params must have precision HERMITE_FP64 and
 * compensated 0; systems outside 2..128 bodies -> E_ARG.
 * hermite_ensemble_init: initial derivatives of every system (as
 * hermite_init), system times, step and record counts reset to 0.
 * hermite_ensemble_run: cfg is a HOST array [n_sys]; each system takes steps
 * until its time reaches cfg.t_end or this call has taken max_steps steps of
 * it.  After every step that ends at t > cfg.rec_from the system's energy
 *   E = sum_i m_i v_i^2 / 2 - sum_{i<j} G m_i m_j (r_ij^2 + eps^2)^(-1/2)
 * is recorded as (t, E) at rec[(sys * rec_cap + k) * 2] (DEVICE buffer, k
 * counting on across calls; beyond rec_cap records are dropped and
 * rec_overflow is set).  E at time 0 is in res.E0.  res (HOST [n_sys])
 * receives every system's time, E0, cumulative steps and records, and flags.
 * Synchronises.  E_NONFINITE if a system's criterion became undefined (its
 * res.failed is 1 and it takes no further steps).
 */
typedef struct {
    double eta;        /* Eq. 25 accuracy parameter, finite and > 0              */
    double t_end;      /* integrate until the system's time reaches t_end       */
    double rec_from;   /* record (t, E) after every step ending past this time  */
    int32_t n_iter;    /* P(EC)^n iterations, 1..64                             */
    int32_t reserved;
} hermite_vstep_cfg;

typedef struct {
    double t;          /* the system's time                                     */
    double E0;         /* its energy at time 0                                  */
    int64_t steps;     /* steps taken since hermite_ensemble_init               */
    int32_t records;   /* records written                                       */
    int32_t failed;    /* 1: the criterion became undefined                     */
    int32_t rec_overflow;
    int32_t reserved;
} hermite_vstep_result;

hermite_status hermite_ensemble_create(const hermite_params *prm, int32_t n_sys, const int64_t *offsets,
                                       void *hip_stream, hermite_ctx **out);
hermite_status hermite_ensemble_init(hermite_ctx *ctx, hermite_state *s);
hermite_status hermite_ensemble_run(hermite_ctx *ctx, hermite_state *s, const hermite_vstep_cfg *cfg,
                                    int64_t max_steps, int32_t rec_cap, double *rec, hermite_vstep_result *res);

/*
 * Launch-shape tuning for hermite_force_derivs.
 *   i_per_thread   1 or 2 i-particles per lane (3 or 4 with the scalar
 *                  source and 4-wave workgroups)
 *   j_split        number of j-ranges summed by separate workgroups (0 = auto,
 *                  1..64; an upper bound: it is reduced to one range per 256 j
 *                  and to what the workspace holds, which is 64 ranges while
 *                  n * 64 <= 4 Mi and at least 4 at any n <= n_max)
 *   j_source       0: j-particles staged through LDS tiles by each workgroup;
 *                  1: j-particles packed once per evaluation into 128-byte
 *                  records and streamed through the scalar unit into SGPRs;
 *                  2: every pair evaluated once for both of its bodies (the
 *                  chain's vectors change sign under i <-> j), with
 *                  i_per_thread 1 and wg_waves 4, j_split ignored; partial
 *                  sums in the context's workspace, added in a fixed order;
 *                  one launch up to 32768 bodies, beyond that one launch per
 *                  pair of chunks of up to 16384 bodies (E_ARG from the
 *                  evaluation if the workspace cannot hold a chunk pair)
 *   wg_waves       4 or 16 wave64 per workgroup; 16 (scalar source and one
 *                  i-particle per lane only): the waves share 64 i-particles
 *                  and split the j-range among themselves, adding their sums
 *                  through LDS, so a modest N needs no j_split
 * E_ARG for values outside these sets.  hermite_autotune times the supported
 * shapes on the given state (which must hold a valid path in s->pred),
 * keeps the fastest and returns it through the non-NULL out pointers.
 */
hermite_status hermite_set_launch(hermite_ctx *ctx, int32_t i_per_thread, int32_t j_split, int32_t j_source,
                                  int32_t wg_waves);
hermite_status hermite_autotune(hermite_ctx *ctx, hermite_state *s, int32_t *i_per_thread, int32_t *j_split,
                                int32_t *j_source, int32_t *wg_waves);

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * evaluation of hermite_force_derivs (every pair once, as launch shape
 * j_source 2 computes it) without a context: a^(0..p) along s->pred into
 * s->eval, p = prm->order/2 - 1, for s->n bodies (s->mass, s->pred [p+1][3][n]
 * and s->eval [p+1][3][n] device pointers; the other state fields are not
 * used).  prm's order, precision, G and eps2 are used (validated as by
 * hermite_create; E_ORDER / E_ARG), n in 0..2^40 (E_ARG beyond).
 * Asynchronous on hip_stream (NULL = null stream).  It allocates nothing: the
 * partial sums live in one 64 MiB device array per GPU, held from the first
 * call on that GPU until the process ends.  One launch covers up to 13056
 * bodies at 8th order (15104 at 6th, 18688 at 4th); more run as pairs of
 * chunks sized to the array, whose results differ from hermite_force_derivs
 * only by the rounding of the partial sums' order.  Calls on one GPU share
 * the array: calls that overlap in time on one GPU (other streams, other
 * threads) race and must be serialised by the caller.  On failure,
 * hermite_last_error(NULL) gives the calling thread's message (E_HIP when
 * the array's address cannot be found or the launch fails).
 */
hermite_status hermite_force_derivs_noalloc(const hermite_params *prm, hermite_state *s, void *hip_stream);

/* Message of the last failed call on ctx ("" if none).  For NULL: the
 * calling thread's last failure of hermite_force_derivs_noalloc, else a
 * static string. */
const char *hermite_last_error(const hermite_ctx *ctx);

/* Library version string. */
const char *hermite_version(void);

/* Device probe (no context): the rate at which the current HIP device
 * completes fused multiply-adds in the accumulating form d = a * b + d that
 * the evaluation's chains use, in lane-FMA per second, in FP64 (precision
 * HERMITE_FP64) or FP32 (HERMITE_MIXED).  Sixteen independent dependent
 * chains per lane, 8192 workgroups of 256 lanes, 2048 iterations, the best
 * of three launches timed with HIP events on a stream of its own (after a
 * warm-up launch); it
 * allocates and frees its own 8 or 16 MiB.  The evaluation's efficiency is
 * quoted against this measured ceiling beside the published peak.  E_ARG for
 * another precision or a NULL out, E_HIP if a HIP call fails. */
hermite_status hermite_fma_rate(int32_t precision, double *lane_fma_per_s);

#ifdef __cplusplus
}
#endif

#endif /* HERMITE_H */
