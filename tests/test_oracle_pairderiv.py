"""Pins of the oracle's pair derivatives (softened force law of Sec. 3 and its
time derivatives) against things that do not share its arithmetic:

* mpmath brute force: 40-digit numerical differentiation of the summed force
  along the polynomial path (tiny N, every order up to 5);
* a circular orbit, where every derivative has a closed form;
* the gradient of the oracle potential (the force is minus its gradient);
* Newton's third law: sum_i m_i a_i^(k) = 0 for every k.
"""
from math import factorial

import mpmath
import numpy as np
import pytest

from oracle import hermite_oracle as ho


def _random_path(rng, n, K, scale=1.0):
    return [rng.normal(size=(3, n)) * scale / (k + 1) for k in range(K + 1)]


def _mp_force_path(mass, path, i, G, eps2):
    n = len(mass)
    K = len(path) - 1
    P = [[[mpmath.mpf(float(path[k][c][j])) for j in range(n)] for c in range(3)] for k in range(K + 1)]
    m = [mpmath.mpf(float(x)) for x in mass]
    e2 = mpmath.mpf(eps2)

    def comp(c):
        def f(t):
            s = mpmath.mpf(0)
            for j in range(n):
                if j == i:
                    continue
                r = [sum((P[k][d][j] - P[k][d][i]) * t ** k / mpmath.factorial(k) for k in range(K + 1))
                     for d in range(3)]
                w = r[0] ** 2 + r[1] ** 2 + r[2] ** 2 + e2
                s += G * m[j] * r[c] * w ** mpmath.mpf(-1.5)
            return s
        return f
    return comp


@pytest.mark.parametrize("eps2", [0.0, 0.3])
def test_brute_force_mpmath(eps2):
    rng = np.random.default_rng(5)
    n, K = 4, 5
    mass = rng.uniform(0.5, 2.0, n)
    path = _random_path(rng, n, K)
    G = 1.3
    out = ho.pair_derivs(mass, path, K=K, G=G, eps2=eps2)
    mpmath.mp.dps = 40
    for i in range(n):
        comp = _mp_force_path(mass, path, i, G, eps2)
        for c in range(3):
            f = comp(c)
            ref = mpmath.diffs(f, 0, K)
            for k, rk in enumerate(ref):
                rk = float(rk)
                assert abs(out[k, c, i] - rk) <= 1e-11 * (abs(rk) + 1e-3 * np.abs(out[k, :, i]).max()), (i, c, k)


def test_circular_orbit_closed_form():
    # Relative path r(t) = R (cos wt, sin wt, 0): every pair derivative is
    # (G m / R^3) r^(n)(t) with r^(n)(0) = R w^n (cos(n pi/2), sin(n pi/2), 0).
    R, om, G, mj = 1.7, 0.8, 1.0, 2.5
    K = 5
    n = 2
    mass = np.array([1.0, mj])
    path = []
    for k in range(K + 1):
        pk = np.zeros((3, n))
        pk[0, 1] = R * om ** k * np.cos(k * np.pi / 2)
        pk[1, 1] = R * om ** k * np.sin(k * np.pi / 2)
        path.append(pk)
    out = ho.pair_derivs(mass, path, K=K, G=G)
    for k in range(K + 1):
        exp = G * mj / R ** 3 * path[k][:, 1]
        assert np.allclose(out[k, :, 0], exp, rtol=0, atol=1e-14 * max(1.0, om ** k))


def test_natural_scale_circular_orbit():
    # On a circular relative orbit every rate |r^(k)|/R equals omega^k, so the
    # natural scale of the k-th derivative is G m / R^2 omega^k exactly; with
    # softening the distance is sqrt(R^2 + eps^2).
    R, om, G, mj, K = 1.7, 0.8, 1.3, 2.5, 5
    mass = np.array([1.0, mj])
    path = []
    for k in range(K + 1):
        pk = np.zeros((3, 2))
        pk[0, 1] = R * om ** k * np.cos(k * np.pi / 2)
        pk[1, 1] = R * om ** k * np.sin(k * np.pi / 2)
        path.append(pk)
    _, nat = ho.pair_derivs(mass, path, K=K, G=G, with_scale=True)
    assert np.allclose(nat[:, 0], [G * mj / R ** 2 * om ** k for k in range(K + 1)], rtol=1e-13)
    eps2 = 0.3
    _, nat = ho.pair_derivs(mass, path, K=K, G=G, eps2=eps2, with_scale=True)
    s = np.sqrt(R * R + eps2)
    rate = [(R * om ** k / s) ** (1.0 / k) for k in range(1, K + 1)]
    ome = max(rate)
    assert np.allclose(nat[:, 0], [G * mj / s ** 2 * ome ** k for k in range(K + 1)], rtol=1e-13)


def test_force_is_minus_gradient_of_potential():
    rng = np.random.default_rng(7)
    n = 6
    mass = rng.uniform(0.1, 1.0, n)
    x = rng.normal(size=(3, n))
    eps2 = 0.01
    a = ho.pair_derivs(mass, [x], K=0, eps2=eps2)[0]
    h = 1e-5
    for i in range(n):
        for c in range(3):
            xp = x.copy(); xp[c, i] += h
            xm = x.copy(); xm[c, i] -= h
            xp2 = x.copy(); xp2[c, i] += 2 * h
            xm2 = x.copy(); xm2[c, i] -= 2 * h
            # potential energy of particle i alone: m_i phi_i; force/m_i = -d phi_i/dx
            f = lambda y: ho.potential_per_particle(mass, y, eps2=eps2)[i]
            d = (-f(xp2) + 8 * f(xp) - 8 * f(xm) + f(xm2)) / (12 * h)
            assert abs(-d - a[c, i]) <= 1e-8 * (1 + abs(a[c, i]))


def test_momentum_all_orders():
    rng = np.random.default_rng(11)
    n, K = 40, 5
    mass = rng.uniform(0.1, 1.0, n)
    path = _random_path(rng, n, K)
    out, mag = ho.pair_derivs(mass, path, K=K, eps2=1e-4, with_mag=True)
    for k in range(K + 1):
        tot = (out[k] * mass).sum(axis=1)
        scale = (mag[k] * mass).sum()
        assert np.all(np.abs(tot) <= 1e-13 * scale)


def test_i_list_subset_matches_full():
    rng = np.random.default_rng(3)
    n = 50
    mass = rng.uniform(0.1, 1.0, n)
    path = _random_path(rng, n, 3)
    full = ho.pair_derivs(mass, path, K=3)
    il = np.array([49, 0, 17, 17, 3])
    sub = ho.pair_derivs(mass, path, K=3, i_list=il)
    assert np.array_equal(sub, full[:, :, il])


def test_self_term_excluded_by_index_and_coincident_nonfinite():
    mass = np.array([1.0, 1.0, 1.0])
    x = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    # particles 0 and 1 coincide: with eps = 0 the result is not finite
    with pytest.raises(ho.NonFiniteError):
        ho.pair_derivs(mass, [x, np.zeros((3, 3))], K=1)
    # with softening it is finite and the coincident pair contributes nothing
    out = ho.pair_derivs(mass, [x, np.zeros((3, 3))], K=1, eps2=1e-6)
    assert np.isfinite(out).all()
    assert out[0, 0, 2] == pytest.approx(-1.0 / (1.0 + 1e-6) ** 1.5 * 2, rel=1e-14)


def test_single_particle_and_empty():
    out = ho.pair_derivs(np.array([1.0]), [np.zeros((3, 1)), np.ones((3, 1))], K=1)
    assert np.array_equal(out, np.zeros((2, 3, 1)))
    out = ho.pair_derivs(np.zeros(0), [np.zeros((3, 0))], K=0)
    assert out.shape == (1, 3, 0)


def test_finite_difference_along_path():
    # Richardson-extrapolated central differences of a(t) evaluated along the
    # polynomial path reproduce a^(1..3) (independent of the derivative chain).
    rng = np.random.default_rng(13)
    n, K = 8, 3
    mass = rng.uniform(0.1, 1.0, n)
    path = _random_path(rng, n, K)
    out = ho.pair_derivs(mass, path, K=K, eps2=0.05)

    def acc_at(t):
        xt = sum(path[k] * t ** k / factorial(k) for k in range(K + 1))
        return ho.pair_derivs(mass, [xt], K=0, eps2=0.05)[0]

    h = 2e-2
    f = {s: acc_at(s * h) for s in range(-4, 5)}
    d1 = (-f[2] + 8 * f[1] - 8 * f[-1] + f[-2]) / (12 * h)
    d2 = (-f[2] + 16 * f[1] - 30 * f[0] + 16 * f[-1] - f[-2]) / (12 * h * h)
    d3 = (-f[3] + 8 * f[2] - 13 * f[1] + 13 * f[-1] - 8 * f[-2] + f[-3]) / (8 * h ** 3)
    for k, d, tol in ((1, d1, 1e-5), (2, d2, 1e-4), (3, d3, 1e-3)):
        scale = np.abs(out[k]).max()
        assert np.abs(d - out[k]).max() <= tol * scale, k
