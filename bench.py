"""Benchmark of the modified Hermite hot path on one MI355X.

Workload: stellar disc of 16384 bodies around a central mass (8th order,
P(EC)^3, dt = 2 pi / 2000; synthetic, seeded).  A timed step is one whole
P(EC)^3 step (predict, 3 x (evaluate a, adot, a^(2), a^(3) ; correct),
interpolate) with the state already in HBM.  Metric: pair interactions per
second, n_iter * N (N - 1) per step, in FP64 and in mixed precision.

Prints ONE JSON line (rank 0, N = 1 GPU only).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLOPS_PER_INTERACTION = {4: 60, 6: 97, 8: 144}
PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3}     # MI355X vector FP64 / FP32 (published)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_mode(precision, w, steps, warmup, autotune=True):
    import torch
    from paper_2006_02501_amd import Hermite

    order, n_iter, dt = w["order"], w["n_iter"], w["dt"]
    n = len(w["mass"])
    h = Hermite(order, n, precision=precision, G=w["G"], eps2=w["eps2"], device="cuda:0")
    st = h.state(w["mass"], w["x"], w["v"])
    h.init(st)
    shape = None
    if autotune:
        h.predict(st, dt)
        shape = h.autotune(st)
    torch.cuda.synchronize()
    E0 = _energy(h, st, w)
    for _ in range(warmup):
        h.step(st, dt, n_iter)
    torch.cuda.synchronize()
    # Timed region: K whole steps.  The evaluation is bracketed by events on
    # the same (torch current) stream the library launches on.
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps * n_iter)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k = 0
    for _ in range(steps):
        h.predict(st, dt)
        for it in range(n_iter):
            evs[k][0].record()
            h.force_derivs(st)
            evs[k][1].record()
            k += 1
            h.correct(st, dt, it == n_iter - 1)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    eval_ms = [a.elapsed_time(b) for a, b in evs]
    E1 = _energy(h, st, w)
    h.close()
    inter = n * (n - 1)
    avg_eval_s = float(np.mean(eval_ms)) / 1e3
    return dict(
        value=steps * n_iter * inter / elapsed,
        ms_per_step=elapsed / steps * 1e3,
        eval_ms_avg=avg_eval_s * 1e3,
        eval_ms_median=float(np.median(eval_ms)),
        eval_interactions_per_s=inter / avg_eval_s,
        launch={"i_per_thread": shape[0], "j_split": shape[1], "j_source": ["lds", "scalar"][shape[2]]}
        if shape else None,
        energy_rel_change=(E1 - E0) / abs(E0),
        flops_per_eval=FLOPS_PER_INTERACTION[order] * inter,
    )


def _energy(h, st, w):
    import torch

    phi = h.potential(st)
    m = st.mass
    kin = 0.5 * torch.sum(m * torch.sum(st.vel * st.vel, dim=0))
    pot = 0.5 * torch.sum(m * phi)
    return float(kin + pot)


def cpu_baseline(w, target_s=12.0):
    """The oracle (plain FP64 C, OpenMP over i) on a bounded sample of the same
    workload: i-particles against all N j-particles, 8th-order derivatives,
    repeated until about target_s seconds of CPU work."""
    from oracle import hermite_oracle as ho

    n = len(w["mass"])
    path = [w["x"], w["v"]]
    acc = ho.pair_derivs(w["mass"], path, K=1)
    path = path + [acc[0], acc[1]]
    rng = np.random.default_rng(7)
    m_i = 64
    while True:
        il = np.sort(rng.choice(n, m_i, replace=False))
        t0 = time.perf_counter()
        ho.pair_derivs(w["mass"], path, K=3, i_list=il)
        dt = time.perf_counter() - t0
        if dt >= target_s / 8 or m_i >= n:
            break
        m_i = min(n, int(m_i * max(2.0, target_s / 8 / max(dt, 1e-3))))
    reps, total = 1, dt
    while total < target_s:
        t0 = time.perf_counter()
        ho.pair_derivs(w["mass"], path, K=3, i_list=il)
        total += time.perf_counter() - t0
        reps += 1
    rate = reps * m_i * (n - 1) / total
    return dict(value=rate, unit="pair interactions/s", cores=ho.num_threads(), kind="oracle",
                sample="%d x (%d random i-particles x all %d j-particles), 8th-order derivatives, %.1f s"
                       % (reps, m_i, n, total))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the kernel at one GPU's share); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch  # noqa: F401
    from workloads import disc16k

    w = disc16k()
    n = len(w["mass"])
    log("bench: disc N=%d order=%d n_iter=%d steps=%d warmup=%d" % (n, w["order"], w["n_iter"], args.steps,
                                                                     args.warmup))
    res = {}
    for prec in ("fp64", "mixed"):
        res[prec] = time_mode(prec, w, args.steps, args.warmup, autotune=not args.no_autotune)
        log("  %s: %.3e interactions/s, %.3f ms/step, eval %.3f ms" % (prec, res[prec]["value"],
                                                                        res[prec]["ms_per_step"],
                                                                        res[prec]["eval_ms_avg"]))
    main_mode = "fp64"
    r = res[main_mode]
    achieved = r["flops_per_eval"] / (r["eval_ms_avg"] / 1e3) / 1e12
    out = {
        "metric": "pair interactions/sec for 8th-order derivs at N=16k: mixed vs FP64, 1 GPU",
        "value": r["value"],
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "disc16k: central mass 1 + 16383 stars of 1e-7, 8th-order modified Hermite, "
                               "P(EC)^3, dt=2pi/2000, G=1, eps=0", "n_bodies": n, "order": 8, "n_iter": 3},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS[main_mode], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS[main_mode], "traffic": None,
                     "kernel": "force_kernel<K=3,FP64> (+ split reduction)",
                     "flops_per_interaction": FLOPS_PER_INTERACTION[8]},
        "modes": {k: {kk: vv for kk, vv in v.items()} for k, v in res.items()},
    }
    mx = res["mixed"]
    mx_ach = mx["flops_per_eval"] / (mx["eval_ms_avg"] / 1e3) / 1e12
    out["modes"]["mixed"]["roofline"] = {"bound": "alu", "achieved": mx_ach, "peak": PEAK_TFLOPS["mixed"],
                                         "unit": "TFLOP/s", "frac": mx_ach / PEAK_TFLOPS["mixed"]}
    out["mixed_over_fp64"] = mx["value"] / r["value"]
    if not args.no_cpu_baseline:
        log("  cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
