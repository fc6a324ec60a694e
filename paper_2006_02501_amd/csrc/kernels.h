// Internal launcher declarations shared by the runtime and the kernel files
// (the evaluation's own are in force_launch.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "force_launch.h"

namespace hermite {

// Predictor and corrector take dt from dt_dev[0] when dt_dev is not null.
hipError_t launch_predict(int p, int64_t n, double dt, const double *dt_dev, const double *pos, const double *vel,
                          const double *deriv, double *pred, hipStream_t st);

// comp: [2][3][n] Kahan compensation of x and v, or null for plain addition.
// dtn_dev (variable step, not last): the next iteration's step length; the
// next path is then the iterate moved from t0 + dt to t0 + dtn_dev[0] along
// its Taylor series.  Null: the iterate itself is the next path.
hipError_t launch_correct(int p, int corrector, int last, int64_t n, double dt, const double *dt_dev,
                          const double *dtn_dev, double *pos, double *vel, double *deriv, const double *eval,
                          double *pred, double *comp, hipStream_t st);

// Time-step criterion (Sec. 3.3): number of workgroup maxima the rate pass
// writes for n particles (and its j-split).
int qmax_partials(int64_t n, int *nsplit, int64_t *j_chunk);

// H = eta q^(-1/2) at x ([3][n], n >= 2) into vs (device double[kVsLen]):
// mode 0: vs[0] = H, vs[slot] = dir H; mode 1: vs[2] = H,
// vs[slot] = dir (vs[0] + H)/2; slot is 1 or 4 (the two step-length slots a
// variable step alternates between); vs[3] = 1 (and vs[slot] = 0) once H is
// not finite and positive.
constexpr int kVsLen = 8;
hipError_t launch_timestep(int64_t n, const double *mass, const double *x, double G, double eps2, double eta,
                           double dir, int mode, int slot, double *qpart, int64_t qpart_cap, double *vs,
                           hipStream_t st);

// The same from count maxima already in qpart (an evaluation with the fused
// pair rate wrote them).
hipError_t launch_timestep_fold(const double *qpart, int count, double eta, double dir, int mode, int slot,
                                double *vs, hipStream_t st);

hipError_t launch_potential(int64_t n, const double *mass, const double *pos, double G, double eps2,
                            double *phi, hipStream_t st);

// flag[0] is set to 1 if any of the count doubles is inf or NaN.
hipError_t launch_check_finite(const double *data, int64_t count, int *flag, hipStream_t st);

// Batched systems ------------------------------------------------------------
struct BatchPlan {
    int32_t n_sys;
    int32_t n_bins;             // 64-lane wavefront bins
    const int32_t *bin_start;   // [n_bins+1] index into bin_sys
    const int32_t *bin_sys;     // systems, bin by bin
    const int64_t *offsets;     // [n_sys+1] particle offsets
    int *counter;               // work counter (device)
};

hipError_t launch_batch_init(const BatchPlan &plan, int p, int64_t n, const double *mass, const double *pos,
                             const double *vel, double *deriv, double G, double eps2, hipStream_t st);

// Launch shape of the batched run kernel.
struct BatchShape {
    int workgroups;   // persistent workgroups (>= 1; at most the bin count is useful)
    int waves;        // wave64 per workgroup, all working on one bin: 1, 2 or 4
    int ring_min;     // bins whose largest system has at least this many bodies
                      // sweep the whole wave as one ring (> 64: never)
};

bool batch_shape_ok(const BatchShape &shape);

// Workgroups of the batched run kernel of this shape (workgroups ignored) a
// CU of the current device holds at once (0 if the query fails).
int batch_resident_per_cu(const BatchShape &shape, int p, bool mixed, bool comp);

// iters: per-system iteration counts (device, [n_sys], each 1..64) or null
// for n_iter everywhere.
// comp: [2][3][n] Kahan compensation of x and v, or null.
hipError_t launch_batch_run(const BatchPlan &plan, int p, bool mixed, int corrector, int64_t n,
                            const double *mass, double *pos, double *vel, double *deriv, const double *dt_sys,
                            int n_steps, int n_iter, const int *iters, double G, double eps2, double *comp,
                            const BatchShape &shape, hipStream_t st);

hipError_t launch_reset_counter(int *counter, hipStream_t st);

// Message of the calling thread's last failed hermite_force_derivs_noalloc
// ("" if none).
const char *noalloc_message();

// Ensemble form (systems of 2..128 bodies, one workgroup each, variable
// time-symmetric steps on the device) -------------------------------------
struct Path6Ptr {
    const double *p[6];
};

// Per-system run settings and running status; their layouts are those of
// hermite_vstep_cfg and hermite_vstep_result in hermite.h.
struct EnsembleCfg {
    double eta, t_end, rec_from;
    int32_t n_iter, reserved;
};
struct EnsembleStatus {
    double t, E0;
    int64_t steps;
    int32_t records, failed, rec_overflow, reserved;
};

struct EnsembleArgs {
    int32_t n_sys;
    int64_t n;                  // bodies over all systems
    const int64_t *offsets;     // [n_sys+1] (device)
    const double *mass;
    double *pos, *vel, *deriv;
    double G, eps2;
    const EnsembleCfg *cfg;     // [n_sys] (device)
    EnsembleStatus *status;     // [n_sys] (device)
    double *rec;                // [n_sys][rec_cap][2] (t, E) (device)
    int32_t rec_cap;
    int64_t max_steps;          // per system and launch
};

hipError_t launch_ensemble_init(const int64_t *offsets, int32_t n_sys, int p, int64_t n, const double *mass,
                                const double *pos, const double *vel, double *deriv, double G, double eps2,
                                hipStream_t st);
hipError_t launch_ensemble_run(const EnsembleArgs &a, int p, int corrector, hipStream_t st);

}  // namespace hermite
