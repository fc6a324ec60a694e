"""Pins of the oracle's corrector coefficients against what the paper fixes.

* Eq. 22-24 (printed correctors) and the beta values quoted with them.
* Eq. 9: the weight of the highest known term F^+-_p in the velocity update.
* Eq. 6, 7, 10, 13: exactness on polynomials and the size of the leading
  truncation terms, checked by integrating polynomials in closed form.
* The standard and Kokubo-Makino 4th-order correctors (Sec. 2.1, Sec. 3.1).
"""
import os
from fractions import Fraction
from math import factorial

import numpy as np
import pytest

from oracle import hermite_oracle as ho

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


@pytest.mark.parametrize("row", _read_golden("position_correctors.txt"), ids=lambda r: "order%s" % r[0])
def test_printed_position_correctors(row):
    order = int(row[0])
    p = order // 2 - 1
    beta = Fraction(row[1])
    assert ho.beta_opt(p) == beta
    printed = [Fraction(c) for c in row[2:]]
    assert ho.endpoint_coefficients(p, beta) == printed


def test_beta_closed_form_values():
    # Eq. 21 evaluated at p = 1, 2, 3 (quoted in Sec. 2.1).
    assert [ho.beta_opt(p) for p in (1, 2, 3)] == [Fraction(11, 3), Fraction(-11, 5), Fraction(163, 35)]


@pytest.mark.parametrize("p", range(1, 7))
def test_eq9_velocity_leading_weight(p):
    # Eq. 9: the coefficient of the p-th term of an order-2(p+1) integrator.
    c = ho.quadrature_weights(p)
    expected = Fraction(1, (-2) ** p) * Fraction(ho.double_factorial(2 * p), ho.double_factorial(2 * p + 1))
    assert c[p] == expected


def test_standard_and_kokubo_makino_4th():
    rows = _read_golden("standard_hermite_4th.txt")
    vel = [r for r in rows if r[0] == "velocity"][0]
    assert ho.endpoint_coefficients(1) == [Fraction(c) for c in vel[2:]]
    for r in rows:
        if r[0] != "position-alpha":
            continue
        alpha = Fraction(r[1])
        coeffs = [Fraction(c) for c in r[2:]]
        # alpha = 1 is beta = 1; alpha = 7/6 is the modified corrector (Sec. 2.1).
        beta = Fraction(1) if alpha == 1 else ho.beta_opt(1)
        assert ho.endpoint_coefficients(1, beta) == coeffs


def test_shifted_corrector_drops_highest_term():
    # beta = 2 - beta_opt removes the F_{2p+2} term's endpoint derivative entirely:
    # the position formula becomes the same-order velocity formula applied to x.
    for p in (1, 2, 3):
        c = ho.endpoint_coefficients(p, ho.corrector_beta(p, "shifted"))
        assert c[-1] == 0
        assert c[:-1] == ho.endpoint_coefficients(p)


def _poly_traj(rng, degree):
    """Random scalar polynomial x(t) = sum c_k t^k; returns coefficient array."""
    return rng.normal(size=degree + 1) / np.array([factorial(k) for k in range(degree + 1)])


def _deriv_at(c, n, t):
    """n-th derivative of the polynomial with coefficients c at t (exact in fp64 up to rounding)."""
    s = 0.0
    for k in range(n, len(c)):
        s += c[k] * factorial(k) / factorial(k - n) * t ** (k - n)
    return s


def _ends(c, p, t0, t1):
    a0 = [np.array([_deriv_at(c, k + 2, t0)]) for k in range(p + 1)]
    a1 = [np.array([_deriv_at(c, k + 2, t1)]) for k in range(p + 1)]
    return a0, a1


@pytest.mark.parametrize("p", [1, 2, 3])
def test_corrector_exact_on_polynomials(p):
    # Eq. 6 with p+1 known derivatives of a at both ends integrates a of degree
    # <= 2p+1 exactly; Eq. 7 with beta = 1 then integrates v of degree <= 2p+2
    # exactly too (x of degree 2p+3).
    rng = np.random.default_rng(10 + p)
    c = _poly_traj(rng, 2 * p + 3)
    t0, dt = 0.3, 0.25
    t1 = t0 + dt
    a0, a1 = _ends(c, p, t0, t1)
    x0 = np.array([_deriv_at(c, 0, t0)])
    v0 = np.array([_deriv_at(c, 1, t0)])
    x1, v1 = ho.correct(p, dt, x0, v0, a0, a1, corrector="beta1")
    assert abs(v1[0] - _deriv_at(c, 1, t1)) <= 1e-13 * (1 + abs(v1[0]))
    assert abs(x1[0] - _deriv_at(c, 0, t1)) <= 1e-13 * (1 + abs(x1[0]))


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("corrector", ["modified", "shifted"])
def test_position_beta_term_eq7_eq13(p, corrector):
    # For x of degree 2p+3 the only position error is the beta term of Eq. 7:
    #   (beta - 1) F_{2p+2} dt / (2p+3),  F_{2p+2} = h^(2p+2)/(2p+2)! v^(2p+2),
    # which Eq. 13 writes as (beta-1)/((2p+3) 2^(p+1)) times the (p+1)-th known
    # term through the diagonal entry 1/2^(p+1) of A^-1.
    rng = np.random.default_rng(20 + p)
    c = _poly_traj(rng, 2 * p + 3)
    t0, dt = -0.2, 0.3
    t1, h = t0 + dt, dt / 2
    a0, a1 = _ends(c, p, t0, t1)
    x0 = np.array([_deriv_at(c, 0, t0)])
    v0 = np.array([_deriv_at(c, 1, t0)])
    beta = float(ho.corrector_beta(p, corrector))
    x1, v1 = ho.correct(p, dt, x0, v0, a0, a1, corrector=corrector)
    F = h ** (2 * p + 2) / factorial(2 * p + 2) * _deriv_at(c, 2 * p + 3, t0 + h)
    expected = (beta - 1.0) / (2 * p + 3) * F * dt
    got = x1[0] - _deriv_at(c, 0, t1)
    assert abs(got - expected) <= 1e-9 * abs(expected) + 1e-15


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_velocity_truncation_eq10(p):
    # Eq. 10: for a of degree 2p+2 the velocity update misses exactly
    #   -1/(-2)^(p+1) (2p+2)!!/(2p+3)!! * 2^(p+1) F_{2p+2} dt
    # (the (p+1)-th known term reduced to F_{2p+2} by the 1/2^(p+1) diagonal of A^-1).
    rng = np.random.default_rng(30 + p)
    c = _poly_traj(rng, 2 * p + 4)           # x degree 2p+4 -> a degree 2p+2
    t0, dt = 0.1, 0.4
    t1, h = t0 + dt, dt / 2
    if p == 0:
        # second-order (trapezoid) velocity update
        a0 = _deriv_at(c, 2, t0); a1 = _deriv_at(c, 2, t1)
        v1 = _deriv_at(c, 1, t0) + 0.5 * (a0 + a1) * dt
    else:
        a0, a1 = _ends(c, p, t0, t1)
        x0 = np.array([_deriv_at(c, 0, t0)])
        v0 = np.array([_deriv_at(c, 1, t0)])
        _, v1 = ho.correct(p, dt, x0, v0, a0, a1)
        v1 = v1[0]
    F = h ** (2 * p + 2) / factorial(2 * p + 2) * _deriv_at(c, 2 * p + 4, t0 + h)
    coef = -Fraction(1, (-2) ** (p + 1)) * Fraction(ho.double_factorial(2 * p + 2),
                                                    ho.double_factorial(2 * p + 3)) * 2 ** (p + 1)
    expected = float(coef) * F * dt
    got = v1 - _deriv_at(c, 1, t1)
    assert abs(got - expected) <= 1e-9 * abs(expected) + 1e-15
