"""Helpers shared by the GPU parity tests (comparison metrics, inputs)."""
import numpy as np

from oracle import hermite_oracle as ho
from workloads import disc16k

TOL_FP64 = 1e-12      # relative bar for FP64 force derivatives, every order

# Mixed precision.  In natural units of a pair (softened distance s, fastest
# rate omega of the relative path, see the oracle's ``with_scale`` output) the
# chain's quantities are bounded by |alpha| <= omega, |beta| <= 3 omega^2,
# |gamma| <= 17 omega^3, hence |r'| <= 1, |J'| <= 4, |S'| <= 34, |C'| <= 466
# (times s omega^k).  One FP32 rounding (u = 2^-24) of terms of that size gives
# the first-order bar u M_k, floored at 1e-6; errors are measured against
# max(|o|, 0.1 S, N_k) with N_k the natural k-th derivative scale.
U32 = 2.0 ** -24
CHAIN_MAGNITUDE = np.array([1.0, 4.0, 34.0, 466.0])
TOL_MIXED = np.maximum(1e-6, U32 * CHAIN_MAGNITUDE)


def within(err, tol):
    """err [K+1][n] against a scalar or per-order tolerance."""
    err = np.asarray(err)
    tol = np.broadcast_to(np.asarray(tol, dtype=np.float64), (max(err.shape[0], 4),))[: err.shape[0]]
    return bool(np.all(err.max(axis=1) <= tol))


def deriv_error(g, o, mag, nat=None):
    """Per particle and derivative order: max-norm error over components divided
    by max(|o|, 0.1 S[, N]), S = sum over j of the pair-term magnitudes (guards
    against cancellation between pairs), N = natural derivative scale (guards
    against cancellation inside a pair's chain; mixed precision only).
    g, o: [K+1][3][n]; mag, nat: [K+1][n].  Returns [K+1][n]."""
    g = np.asarray(g)
    o = np.asarray(o)
    num = np.abs(g - o).max(axis=1)
    den = np.maximum(np.sqrt((o * o).sum(axis=1)), 0.1 * np.asarray(mag))
    if nat is not None:
        den = np.maximum(den, np.asarray(nat))
    den = np.where(den > 0, den, 1.0)
    return num / den


def disc_path(n, p, seed_shift=0):
    """Disc workload of n bodies with a realistic evaluation path x, v, a, adot
    (a and adot exact from the oracle)."""
    w = disc16k(n)
    path = [w["x"], w["v"]]
    if p >= 2:
        out = ho.pair_derivs(w["mass"], path, K=1)
        path = path + [out[0], out[1]][: p - 1]
    return w, path


def random_path(rng, n, p, spread=1.0):
    mass = rng.uniform(0.5, 1.5, n) / max(n, 1)
    path = [rng.normal(size=(3, n)) * spread / (k + 1) for k in range(p + 1)]
    return mass, path


def rel_max(g, o):
    g = np.asarray(g)
    o = np.asarray(o)
    scale = np.abs(o).max()
    return float(np.abs(g - o).max() / (scale if scale > 0 else 1.0))
