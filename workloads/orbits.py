"""Keplerian orbital elements -> Cartesian state (input generation only)."""
import numpy as np


def solve_kepler(M, e, tol=1e-15, max_iter=100):
    """Eccentric anomaly E with E - e sin E = M (Newton's method, vectorised)."""
    M = np.asarray(M, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    M = np.mod(M, 2 * np.pi)
    E = np.where(e < 0.8, M, np.pi * np.ones_like(M))
    for _ in range(max_iter):
        f = E - e * np.sin(E) - M
        dE = f / (1.0 - e * np.cos(E))
        E = E - dE
        if np.all(np.abs(dE) <= tol * np.maximum(1.0, np.abs(E))):
            break
    return E


def elements_to_cartesian(mu, a, e, inc, node, peri, mean_anom):
    """Relative position and velocity [3][n] for bound orbits (e < 1).

    mu = G (M + m); angles in radians; the reference plane is xy.
    """
    mu, a, e, inc, node, peri, mean_anom = np.broadcast_arrays(
        *[np.asarray(q, dtype=np.float64) for q in (mu, a, e, inc, node, peri, mean_anom)])
    E = solve_kepler(mean_anom, e)
    cE, sE = np.cos(E), np.sin(E)
    b = np.sqrt(1.0 - e * e)
    xq = a * (cE - e)
    yq = a * b * sE
    nmot = np.sqrt(mu / a ** 3)
    Edot = nmot / (1.0 - e * cE)
    vxq = -a * sE * Edot
    vyq = a * b * cE * Edot
    cO, sO = np.cos(node), np.sin(node)
    cw, sw = np.cos(peri), np.sin(peri)
    ci, si = np.cos(inc), np.sin(inc)
    # Rotation Rz(node) Rx(inc) Rz(peri) applied to the perifocal frame.
    P = np.stack([cO * cw - sO * sw * ci, sO * cw + cO * sw * ci, sw * si])
    Q = np.stack([-cO * sw - sO * cw * ci, -sO * sw + cO * cw * ci, cw * si])
    r = P * xq + Q * yq
    v = P * vxq + Q * vyq
    return r, v


def to_barycentric(mass, x, v):
    """Shift positions and velocities so the centre of mass is at rest at the origin."""
    mass = np.asarray(mass, dtype=np.float64)
    mt = mass.sum()
    xc = (x * mass).sum(axis=1, keepdims=True) / mt
    vc = (v * mass).sum(axis=1, keepdims=True) / mt
    return x - xc, v - vc
