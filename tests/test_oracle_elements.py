"""Pins of the oracle's orbital-element diagnostic, ``kepler_elements``.

It returns the eccentricity vector (Appendix A, first equation: the
Laplace-Runge-Lenz vector divided by mu), its length, and the argument of
periapsis whose drift Sec. 3.1 follows.  Nothing here calls the oracle's own
element arithmetic to build an expectation.  Each orbit is built in closed form
from known elements:

* a semi-major axis a, an eccentricity e, an inclination i, a node Omega, an
  argument of periapsis omega and a true anomaly f;
* perifocal unit vectors P and Q, rotated by R_z(Omega) R_x(i) R_z(omega);
* r = p / (1 + e cos f) (cos f P + sin f Q) and
  v = sqrt(mu / p) (-sin f P + (e + cos f) Q), with p = a (1 - e^2).

The eccentricity vector of that orbit is e P.  Its argument of periapsis is:

* omega itself, measured from the ascending node, for an inclined orbit;
* the longitude of periapsis Omega + omega from +x, for a prograde orbit in
  the xy-plane (there is no node);
* the angle of P from +x taken in the sense of the motion, omega - Omega, for
  a retrograde orbit in the xy-plane.

Exact Kepler motion, from 30-digit solutions of Kepler's equation, must
leave e and omega unchanged at every phase.  The planted mistakes these
tests catch include:

* a wrong sign in either term of the vector;
* mu without the orbiting body's mass;
* a node vector of the wrong sign;
* a dropped retrograde flip;
* the orbiting body taken relative to the origin rather than to the central
  body.
"""
import mpmath
import numpy as np
import pytest

from oracle import hermite_oracle as ho


def _rot_z(t):
    c, s = np.cos(t), np.sin(t)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def _rot_x(t):
    c, s = np.cos(t), np.sin(t)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def _perifocal(inc, node, argp):
    m = _rot_z(node) @ _rot_x(inc) @ _rot_z(argp)
    return m[:, 0], m[:, 1]


def _relative_state(mu, a, e, inc, node, argp, f):
    """Relative position and velocity of a Kepler orbit from its elements."""
    P, Q = _perifocal(inc, node, argp)
    p = a * (1.0 - e * e)
    r = p / (1.0 + e * np.cos(f))
    x = r * (np.cos(f) * P + np.sin(f) * Q)
    v = np.sqrt(mu / p) * (-np.sin(f) * P + (e + np.cos(f)) * Q)
    return x, v, P


def _two_body(m_c, m_k, G, rel_x, rel_v, shift=None, boost=None, extra=0):
    """Bodies [c, k] (plus `extra` far, unrelated bodies) with the given relative
    orbit of k about c, the central body placed at `shift`, moving with `boost`."""
    n = 2 + extra
    mass = np.concatenate([[m_c, m_k], np.full(extra, 0.5)])
    x = np.zeros((3, n))
    v = np.zeros((3, n))
    s = np.zeros(3) if shift is None else np.asarray(shift, float)
    b = np.zeros(3) if boost is None else np.asarray(boost, float)
    x[:, 0], v[:, 0] = s, b
    x[:, 1], v[:, 1] = s + rel_x, b + rel_v
    for q in range(extra):
        x[:, 2 + q] = [40.0 + 7 * q, -30.0, 5.0 * q]
        v[:, 2 + q] = [0.1, 0.2 * q, -0.3]
    return mass, x, v


def _ang(d):
    return abs(np.angle(np.exp(1j * d)))


# (a, e, i, Omega, omega): inclined orbits with a node, of either sense (i < or > pi/2)
INCLINED = [
    (1.0, 0.1, 0.3, 1.1, 0.7),
    (2.5, 0.5, 1.2, -2.0, 2.9),
    (0.3, 0.05, 0.02, 4.0, -1.3),
    (1.7, 0.8, 2.4, 0.4, 5.5),       # retrograde but inclined: still measured from the node
    (1.0, 0.3, np.pi / 2, 2.2, 0.1),  # polar
]


@pytest.mark.parametrize("elem", INCLINED)
@pytest.mark.parametrize("f", [0.0, 1.3, np.pi, 4.4])
def test_inclined_orbit_elements(elem, f):
    a, e, inc, node, argp = elem
    m_c, m_k, G = 1.0, 0.3, 2.0          # a heavy companion: mu must include it
    mu = G * (m_c + m_k)
    rx, rv, P = _relative_state(mu, a, e, inc, node, argp, f)
    mass, x, v = _two_body(m_c, m_k, G, rx, rv)
    ev, en, om = ho.kepler_elements(mass, x, v, 1, 0, G=G)
    assert np.max(np.abs(ev - e * P)) < 2e-14 * max(1.0, a)
    assert abs(en - e) < 2e-14
    assert _ang(om - argp) < 1e-12 / e


@pytest.mark.parametrize("e", [0.05, 0.4, 0.9])
@pytest.mark.parametrize("node,argp", [(0.0, 0.8), (1.9, -2.4), (3.0, 3.0)])
def test_planar_prograde_longitude_of_periapsis(e, node, argp):
    mu = 1.0 + 1e-3
    rx, rv, P = _relative_state(mu, 1.0, e, 0.0, node, argp, 2.1)
    mass, x, v = _two_body(1.0, 1e-3, 1.0, rx, rv)
    ev, en, om = ho.kepler_elements(mass, x, v, 1)
    assert np.max(np.abs(ev - e * P)) < 2e-14
    assert abs(en - e) < 2e-14
    assert _ang(om - (node + argp)) < 1e-13 / e


@pytest.mark.parametrize("e", [0.05, 0.4, 0.9])
@pytest.mark.parametrize("node,argp", [(0.0, 0.8), (1.9, -2.4)])
def test_planar_retrograde_angle_in_sense_of_motion(e, node, argp):
    mu = 1.0 + 1e-3
    rx, rv, P = _relative_state(mu, 1.0, e, np.pi, node, argp, 0.6)
    # the orbit runs clockwise seen from +z
    assert np.cross(rx, rv)[2] < 0
    mass, x, v = _two_body(1.0, 1e-3, 1.0, rx, rv)
    ev, en, om = ho.kepler_elements(mass, x, v, 1)
    assert np.max(np.abs(ev - e * P)) < 2e-14
    # P lies at angle Omega - omega from +x counterclockwise, i.e. at
    # omega - Omega in the sense of the motion
    assert _ang(om - (argp - node)) < 1e-13 / e


def test_frame_and_body_index_independence():
    """Elements of body k about body c do not depend on where the pair sits,
    how it moves, their indices among other bodies, or the other bodies."""
    a, e, inc, node, argp = INCLINED[1]
    G, m_c, m_k = 1.0, 1.0, 1e-3
    rx, rv, P = _relative_state(G * (m_c + m_k), a, e, inc, node, argp, 0.9)
    mass, x, v = _two_body(m_c, m_k, G, rx, rv, shift=[3.0, -7.0, 11.0], boost=[0.4, -0.2, 0.9], extra=3)
    perm = np.array([3, 1, 4, 0, 2])   # body c ends at index 3, body k at index 1
    mass, x, v = mass[perm], x[:, perm], v[:, perm]
    ev, en, om = ho.kepler_elements(mass, x, v, 1, 3, G=G)
    assert np.max(np.abs(ev - e * P)) < 1e-13
    assert _ang(om - argp) < 1e-12


def _kepler_state_mp(mu, a, e, inc, node, argp, M0, t):
    """Relative state at time t of an exact Kepler orbit (30 digits), rounded."""
    with mpmath.workdps(30):
        n = mpmath.sqrt(mpmath.mpf(mu) / mpmath.mpf(a) ** 3)
        M = mpmath.mpf(M0) + n * mpmath.mpf(t)
        E = mpmath.findroot(lambda E: E - e * mpmath.sin(E) - M, M)
        f = 2 * mpmath.atan2(mpmath.sqrt(1 + e) * mpmath.sin(E / 2), mpmath.sqrt(1 - e) * mpmath.cos(E / 2))
        p = mpmath.mpf(a) * (1 - mpmath.mpf(e) ** 2)
        r = p / (1 + e * mpmath.cos(f))
        cn, sn = mpmath.cos(node), mpmath.sin(node)
        ci, si = mpmath.cos(inc), mpmath.sin(inc)
        cw, sw = mpmath.cos(argp), mpmath.sin(argp)
        P = [cn * cw - sn * ci * sw, sn * cw + cn * ci * sw, si * sw]
        Q = [-cn * sw - sn * ci * cw, -sn * sw + cn * ci * cw, si * cw]
        k = mpmath.sqrt(mpmath.mpf(mu) / p)
        x = [r * (mpmath.cos(f) * P[c] + mpmath.sin(f) * Q[c]) for c in range(3)]
        v = [k * (-mpmath.sin(f) * P[c] + (e + mpmath.cos(f)) * Q[c]) for c in range(3)]
        return np.array([float(q) for q in x]), np.array([float(q) for q in v])


@pytest.mark.parametrize("elem", [INCLINED[0], INCLINED[3], (1.0, 0.5, 0.0, 0.7, 1.9)])
def test_constant_along_exact_kepler_motion(elem):
    a, e, inc, node, argp = elem
    G, m_c, m_k = 1.0, 1.0, 1e-3
    mu = G * (m_c + m_k)
    period = 2 * np.pi * np.sqrt(a ** 3 / mu)
    es, oms = [], []
    for t in np.linspace(0.0, 1.3 * period, 11):
        rx, rv = _kepler_state_mp(mu, a, e, inc, node, argp, 0.4, t)
        mass, x, v = _two_body(m_c, m_k, G, rx, rv)
        ev, en, om = ho.kepler_elements(mass, x, v, 1)
        es.append(ev)
        oms.append(om)
    es = np.array(es)
    assert np.max(np.abs(es - es[0])) < 5e-14
    assert max(_ang(o - oms[0]) for o in oms) < 1e-12 / e
    expect = argp if inc != 0.0 else node + argp
    assert _ang(oms[0] - expect) < 1e-12 / e


def test_wrap_angle_range():
    for d, want in [(0.0, 0.0), (np.pi, np.pi), (-np.pi, np.pi), (3 * np.pi, np.pi), (2 * np.pi + 0.1, 0.1),
                    (-2 * np.pi - 0.1, -0.1), (7.0, 7.0 - 2 * np.pi)]:
        got = ho.wrap_angle(d)
        assert -np.pi < got <= np.pi
        assert abs(got - want) < 1e-12


@pytest.mark.parametrize("elem", [INCLINED[0], INCLINED[3]])
@pytest.mark.parametrize("eps2", [0.0, 1e-6])
def test_energy_two_body_closed_form(elem, eps2):
    """The energy diagnostic of Sec. 3.1 for two bodies in their barycentric
    frame: without softening it is -G m_c m_k / (2 a), the vis-viva energy
    of the relative orbit times the reduced mass; with softening the potential
    term is -G m_c m_k (r^2 + eps^2)^(-1/2)."""
    a, e, inc, node, argp = elem
    G, m_c, m_k = 1.5, 1.0, 0.2
    mu = G * (m_c + m_k)
    for f in (0.0, 2.0, 4.0):
        rx, rv, _ = _relative_state(mu, a, e, inc, node, argp, f)
        mass = np.array([m_c, m_k])
        x = np.stack([-m_k / (m_c + m_k) * rx, m_c / (m_c + m_k) * rx], axis=1)
        v = np.stack([-m_k / (m_c + m_k) * rv, m_c / (m_c + m_k) * rv], axis=1)
        got = ho.energy(mass, x, v, G=G, eps2=eps2)
        r = np.sqrt(rx @ rx)
        want = -G * m_c * m_k / (2 * a) + G * m_c * m_k * (1.0 / r - 1.0 / np.sqrt(r * r + eps2))
        assert abs(got - want) < 1e-14 * abs(want)
