"""Pins of the oracle's variable time-symmetric step (Sec. 3.3, Eq. 25).

The criterion H(x) is pinned by Kepler's third law (for two bodies it is eta
times the orbital period over 2 pi), by its scaling and invariance, and by the
minimum over pairs; the step built on it by reversibility (a converged step
taken backwards returns to its start and has the same length), by the
constant step length of a circular orbit, by the order of the energy error
in eta, by the energy error returning to round-off after whole orbits, by the
trends of the paper's disc test (Table 1), and by the Taylor shift that moves
an iterate to a new end point."""
import math

import numpy as np
import pytest

from oracle import hermite_oracle as ho
from workloads import disc100, kepler_two_body


def _two_body(sep, m1, m2):
    mass = np.array([m1, m2])
    x = np.zeros((3, 2))
    x[0, 1] = sep
    return mass, x


def test_criterion_is_kepler_period_for_two_bodies():
    # Kepler's third law: a circular binary of separation d has period
    # T = 2 pi sqrt(d^3 / (G (m1 + m2))), so H = eta T / (2 pi).
    for sep, m1, m2, G in ((2.0, 1.0, 1e-3, 1.0), (0.37, 3.0, 0.5, 2.5), (15.0, 1e-5, 1e-5, 1.0)):
        mass, x = _two_body(sep, m1, m2)
        period = 2.0 * math.pi * math.sqrt(sep ** 3 / (G * (m1 + m2)))
        H = ho.step_criterion(mass, x, 0.1, G=G)
        assert H == pytest.approx(0.1 * period / (2.0 * math.pi), rel=1e-15)


def test_criterion_scaling_and_invariance():
    rng = np.random.default_rng(7)
    n = 17
    mass = rng.uniform(0.1, 2.0, n)
    x = rng.normal(size=(3, n))
    eps2 = 1e-3
    H = ho.step_criterion(mass, x, 0.05, eps2=eps2)
    # lengths x L (softening too): H x L^(3/2); masses x M: H x M^(-1/2)
    assert ho.step_criterion(mass, 4.0 * x, 0.05, eps2=16.0 * eps2) == pytest.approx(8.0 * H, rel=1e-14)
    assert ho.step_criterion(9.0 * mass, x, 0.05, eps2=eps2) == pytest.approx(H / 3.0, rel=1e-14)
    assert ho.step_criterion(mass, x, 0.1, eps2=eps2) == pytest.approx(2.0 * H, rel=1e-15)
    # translation, rotation about z and relabelling change nothing
    c, s = math.cos(0.7), math.sin(0.7)
    R = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    perm = rng.permutation(n)
    assert ho.step_criterion(mass, x + np.array([[3.0], [-1.0], [0.5]]), 0.05, eps2=eps2) == pytest.approx(H, rel=1e-12)
    assert ho.step_criterion(mass, R @ x, 0.05, eps2=eps2) == pytest.approx(H, rel=1e-12)
    assert ho.step_criterion(mass[perm], x[:, perm], 0.05, eps2=eps2) == H
    # softening only lengthens the step
    assert ho.step_criterion(mass, x, 0.05, eps2=0.0) < H


def test_criterion_takes_the_tightest_pair():
    # a binary (d = 0.01) plus a far third body: H is the binary's; moving the
    # third body closer to the heavier member than any other pair takes over.
    mass = np.array([1.0, 1e-3, 0.2])
    x = np.zeros((3, 3))
    x[0, 1] = 0.01
    x[0, 2] = 50.0
    kep = lambda d, m: 0.1 * math.sqrt(d ** 3 / m)
    assert ho.step_criterion(mass, x, 0.1) == pytest.approx(kep(0.01, 1.001), rel=1e-14)
    x[1, 2], x[0, 2] = 0.002, 0.0
    assert ho.step_criterion(mass, x, 0.1) == pytest.approx(kep(0.002, 1.2), rel=1e-14)
    # fewer than two bodies: no pair, no step
    with pytest.raises(ValueError):
        ho.step_criterion(mass[:1], x[:, :1], 0.1)


def _kepler_state(order, e, M=0.3):
    k = kepler_two_body(e=e, mean_anomaly=M)
    st = ho.State(k["mass"], k["x"], k["v"], order // 2 - 1)
    ho.init_derivs(st)
    return k, st


@pytest.mark.parametrize("order", [4, 6, 8])
def test_circular_orbit_takes_constant_step(order):
    # a circular orbit keeps its separation (to the scheme's accuracy: 1e-8
    # relative at 4th order here), so every step is H itself
    k, st = _kepler_state(order, 0.0)
    eta = 0.05
    H = eta * k["period"] / (2.0 * math.pi)
    for _ in range(20):
        dt = ho.step_symmetric(st, eta, 4)
        assert dt == pytest.approx(H, rel=1e-6)
    assert st.t == pytest.approx(20 * H, rel=1e-6)


@pytest.mark.parametrize("order", [4, 6, 8])
def test_converged_step_is_reversible(order):
    # e = 0.7 away from apsides: H changes by ~10 % over one step.  Taken to
    # convergence, a step backwards from the end lands on the start and has
    # the same length.
    k, st = _kepler_state(order, 0.7, M=0.4)
    x0, v0 = st.x.copy(), st.v.copy()
    dt_f = ho.step_symmetric(st, 0.1, 12)
    dt_b = ho.step_symmetric(st, 0.1, 12, direction=-1.0)
    assert dt_b == pytest.approx(-dt_f, rel=1e-13)
    assert abs(ho.step_criterion(k["mass"], x0, 0.1) / dt_f - 1.0) > 0.02
    assert np.max(np.abs(st.x - x0)) < 1e-13 and np.max(np.abs(st.v - v0)) < 1e-13
    assert abs(st.t) < 1e-15


def test_start_of_step_criterion_alone_is_not_reversible():
    # the same step with dt = H(start) only (no symmetrisation) does not
    # return: the backward step starts from H(end) instead.
    k, st = _kepler_state(8, 0.7, M=0.4)
    x0 = st.x.copy()
    ho.step(st, ho.step_criterion(st.mass, st.x, 0.1), 12)
    ho.step(st, -ho.step_criterion(st.mass, st.x, 0.1), 12)
    assert np.max(np.abs(st.x - x0)) > 1e-4


def _kepler_energy_run(order, eta, n_iter, periods, e=0.5):
    k, st = _kepler_state(order, e, M=0.0)
    E0 = ho.energy(st.mass, st.x, st.v)
    worst = 0.0
    while st.t < periods * k["period"] * (1.0 - 1e-9):
        ho.step_symmetric(st, eta, n_iter)
        worst = max(worst, abs(ho.energy(st.mass, st.x, st.v) / E0 - 1.0))
    return worst, abs(ho.energy(st.mass, st.x, st.v) / E0 - 1.0), st


@pytest.mark.parametrize("order,eta", [(4, 0.04), (6, 0.04), (8, 0.16)])
def test_energy_error_order_in_eta(order, eta):
    # converged iterations: the largest energy error over one orbit scales
    # as eta^order
    w1, _, _ = _kepler_energy_run(order, eta, 8, 1)
    w2, _, _ = _kepler_energy_run(order, eta / 2, 8, 1)
    ratio = w1 / w2
    assert 0.7 * 2 ** order < ratio < 1.4 * 2 ** order, ratio


def test_energy_error_returns_after_whole_orbits():
    # time symmetry: the energy error made during an orbit is undone over
    # the rest of it (no secular term), so after 3 whole orbits it sits far
    # below its largest value in between
    worst, last, st = _kepler_energy_run(4, 0.04, 8, 3)
    assert worst > 1e-8
    assert last < 1e-4 * worst


@pytest.fixture(scope="module")
def disc_runs():
    # the disc of the paper's N-body test (Sec. 3.3), run for one time unit;
    # statistic: median |E/E0 - 1| over the last half unit
    w = disc100()
    out = {}
    for order, eta, n_iter in ((8, 0.16, 1), (8, 0.16, 2), (8, 0.16, 3), (8, 0.16, 4), (8, 0.08, 3), (4, 0.08, 3)):
        st = ho.State(w["mass"], w["x"], w["v"], order // 2 - 1)
        ho.init_derivs(st, eps2=w["eps2"])
        E0 = ho.energy(st.mass, st.x, st.v, eps2=w["eps2"])
        rec = []
        while st.t < 1.0:
            ho.step_symmetric(st, eta, n_iter, eps2=w["eps2"])
            rec.append((st.t, abs(ho.energy(st.mass, st.x, st.v, eps2=w["eps2"]) / E0 - 1.0)))
        rec = np.array(rec)
        out[(order, eta, n_iter)] = np.median(rec[rec[:, 0] > 0.5, 1])
    return out


def test_disc_table1_trends(disc_runs):
    d = disc_runs
    # Every correction takes the end values at the end of the step it makes,
    # so the iteration settles fast: n = 2, 3 and 4 give the same error (a
    # correction with an updated dt but the end values of the previous end
    # point gains only a factor of a few hundred per iteration here).
    e2, e3, e4 = d[(8, 0.16, 2)], d[(8, 0.16, 3)], d[(8, 0.16, 4)]
    assert abs(e3 / e2 - 1.0) < 0.1 and abs(e4 / e3 - 1.0) < 0.1, (e2, e3, e4)
    # n = 1 (one correction, no iterate to take H_+ from after it) is far
    # worse (Sec. 3.1's n-sweep discussion)
    assert d[(8, 0.16, 1)] > 1e3 * e2
    # halving eta gains more than the 2^8 of the order (down to round-off)
    assert d[(8, 0.08, 3)] < e3 / 2.0 ** 8
    # the 4th-order scheme at the same eta and n is far less accurate
    assert d[(4, 0.08, 3)] > 1e3 * d[(8, 0.08, 3)]


def test_symmetric_step_rejects_bad_arguments():
    k, st = _kepler_state(4, 0.5)
    with pytest.raises(ValueError):
        ho.step_symmetric(st, 0.1, 0)


def test_shift_iterate_is_the_taylor_series_of_a_polynomial_path():
    # a path that is a polynomial of degree p + 2 in t is moved exactly: its
    # derivatives at t1 + d are those of the polynomial there
    rng = np.random.default_rng(3)
    for p in (1, 2, 3):
        deg = p + 2
        c = rng.normal(size=(deg + 1, 3, 5))      # x(t) = sum_q c_q t^q
        def deriv(f, t):
            return sum(c[q] * (math.factorial(q) / math.factorial(q - f)) * t ** (q - f)
                       for q in range(f, deg + 1))
        t1, d = 0.3, -0.07
        x1, v1 = deriv(0, t1), deriv(1, t1)
        a1 = [deriv(k + 2, t1) for k in range(p + 1)]
        path = ho.shift_iterate(p, d, x1, v1, a1)
        assert len(path) == p + 1
        for f in range(p + 1):
            assert np.allclose(path[f], deriv(f, t1 + d), rtol=1e-13, atol=1e-13), (p, f)
        # no move: the iterate itself
        same = ho.shift_iterate(p, 0.0, x1, v1, a1)
        assert all(np.array_equal(same[f], ([x1, v1] + a1)[f]) for f in range(p + 1))
