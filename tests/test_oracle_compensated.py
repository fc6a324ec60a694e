"""Pins of compensated summation in the oracle's time integration (Sec. 3.2,
reading R22): Kahan's textbook case, a free particle whose exact position is
known in rational arithmetic, and the round-off-limited 8th-order Kepler
energy error the paper reduces with it."""
from fractions import Fraction

import numpy as np

from oracle import hermite_oracle as ho
from workloads import kepler_two_body


def test_kahan_add_recovers_lost_increments():
    # 1 + 10^4 x 1e-16: plain addition loses every increment (each is below
    # half an ulp of 1); the compensated sum is the exact sum rounded once.
    s, c = 1.0, 0.0
    plain = 1.0
    for _ in range(10000):
        s, c = ho.kahan_add(s, c, 1e-16)
        plain += 1e-16
    exact = Fraction(1) + 10000 * Fraction(1e-16)
    assert plain == 1.0
    assert abs(Fraction(s) - exact) <= Fraction(np.spacing(1.0)) / 2
    # the compensation holds what the sum cannot represent
    assert abs(Fraction(s) - Fraction(c) - exact) < abs(Fraction(s) - exact) or Fraction(s) == exact


def _free_particle(compensated, steps=10000, dt=0.1):
    st = ho.State([1.0], [[0.7], [0.0], [0.0]], [[1.0 / 3.0], [0.0], [0.0]], 1)
    ho.init_derivs(st)
    for _ in range(steps):
        ho.step(st, dt, 1, compensated=compensated)
    # with a = 0 every step adds fl(v dt) exactly once (weight 1 on (v0+v1)/2)
    inc = Fraction(float(np.float64(1.0 / 3.0) * dt))
    exact_x = Fraction(0.7) + steps * inc
    return st, abs(Fraction(float(st.x[0, 0])) - exact_x), abs(Fraction(st.t) - steps * Fraction(dt))


def test_free_particle_position_and_time():
    st_c, err_c, terr_c = _free_particle(True)
    st_p, err_p, terr_p = _free_particle(False)
    ulp = Fraction(float(np.spacing(st_c.x[0, 0])))
    # compensated: within one ulp of the exact sum of the increments, and the
    # time exact; plain summation drifts by hundreds of ulp
    assert err_c <= ulp
    assert terr_c <= Fraction(float(np.spacing(st_c.t)))
    assert err_p > 50 * ulp
    assert terr_p > 100 * Fraction(float(np.spacing(st_p.t)))
    # the velocity never changes
    assert st_c.v[0, 0] == 1.0 / 3.0 and np.all(st_c.cv == 0.0)


def _kepler_worst_energy(compensated, orbits=4, dt=2.0 ** -5):
    k = kepler_two_body(e=0.1)
    st = ho.State(k["mass"], k["x"], k["v"], 3)
    ho.init_derivs(st, eps2=1e-16)
    E0 = ho.energy(st.mass, st.x, st.v, eps2=1e-16)
    worst = 0.0
    for _ in range(int(orbits * 2 * np.pi / dt)):
        ho.step(st, dt, 3, eps2=1e-16, compensated=compensated)
        worst = max(worst, abs(ho.energy(st.mass, st.x, st.v, eps2=1e-16) / E0 - 1.0))
    return worst


def test_compensation_lowers_round_off_energy_error():
    # Sec. 3.2: at a step where the 8th-order truncation error is below
    # double-precision round-off (Kepler, e = 0.1, dt = 2^-5), compensated
    # summation lowers the energy error (4 orbits; ~3x here)
    plain = _kepler_worst_energy(False)
    comp = _kepler_worst_energy(True)
    assert plain < 1e-14
    assert comp < 0.5 * plain
