"""ORACLE -- test infrastructure only.

A plain, slow, FP64 CPU implementation of the modified Hermite integrators of
Dittmann (2020), "Modified Hermite Integrators of Arbitrary Order"
(arXiv:2006.02501).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with the
HIP path under ``paper_2006_02501_amd/``; the only thing both sides use is the
seeded initial-condition generator in ``workloads/``.

What each function follows (section / equation of the paper):

* ``beta_opt``             Eq. 21 (closed form of the optimal beta).
* ``even_pascal_matrix``   Eq. 8 (A_{n,m} = C(2m, n)).
* ``quadrature_weights``   Eq. 6 (velocity, even terms up to F_2p) and Eq. 7
                           (position, one more even term weighted by beta),
                           with the unknown even terms F_0, F_2, ... obtained
                           from the known F^+-_n by solving Eq. 8 exactly in
                           rational arithmetic.
* ``correct``              Eq. 4-8: form F^+-_n (Eq. 5) from the derivatives
                           at both ends of the step (h = dt/2, Eq. 1), apply the
                           Eq. 6 weights to get v1 first, then the Eq. 7 weights
                           with f = v (its derivatives being a, adot, ...) to
                           get x1, as Sec. 2 requires (velocity first).
* ``predict``              Sec. 3, second paragraph: standard Taylor series
                           using every stored derivative of a.
* ``pair_derivs``          Sec. 3 opening paragraph: softened force law and its
                           time derivatives (C part, ``pairderiv.c``).
* ``init_derivs``          Sec. 3, second paragraph: explicit higher
                           derivatives at t0 (up to a^(5) at 8th order).
* ``interpolate_higher``   Reading R2 below: a^(p+1..2p-1) at the end of a step
                           from the Hermite interpolant through a^(0..p) at both
                           ends, solved numerically (confluent Vandermonde).
* ``step``                 Sec. 2 end / Sec. 3: P(EC)^n iteration.
* ``kahan_add``            Sec. 3.2: compensated summation (reading R22).
* ``step_criterion``,      Sec. 3.3, Eq. 25: the minimum two-body time scale
  ``step_symmetric``,      and the implicit time-symmetric step (reading R21),
  ``shift_iterate``        whose iterates move to each new end point along their
                           own Taylor series.
* ``energy``, ``kepler_elements``  Sec. 3.1 diagnostics; eccentricity vector of
                           Appendix A (first equation).

Readings where the paper is silent (frozen identically in the HIP path):
  R1  the predictor uses all stored derivatives a^(0..2p-1): x to dt^(2p+1),
      v to dt^(2p); the predicted a (and adot) feed the 6th/8th-order pair
      terms.
  R2  a^(p+1..2p-1) at the end of a step come from the Hermite interpolant.
  R3  P(EC)^n iteration k >= 2 evaluates at the corrected (x1, v1) with the
      relative a, adot taken from iteration k-1's evaluation.
  R6  the self term is excluded by index, never by distance.
  R21 variable step (Sec. 3.3): H_- at the start of the step; a first
      prediction with dt = H_- gives H_+ at its end point and dt_1 =
      (H_- + H_+)/2, and the prediction is redone for dt_1.  Every iteration
      corrects with the dt whose end point it evaluated (the corrector's end
      values belong to t0 + dt, Eq. 4-8); H_+ at that evaluation point gives
      the next dt, and the iterate is moved to the new end point along its own
      Taylor series.  Converged iterations give the time-symmetric step.
  R22 compensated summation (Sec. 3.2, for the time integration): x, v and t
      each carry a Kahan compensation term; the corrector adds its increments
      dv, dx (and the step adds dt) through it.  Every iterate of a step uses
      the carried terms; the last iteration stores the new ones.  They are
      part of the state (zero at the start).

Parity pins for every function are in ``tests/test_oracle_*.py``.
"""
from fractions import Fraction
from math import comb, factorial
import ctypes
import os

import numpy as np

from . import build as _build

# ----------------------------------------------------------------------------
# Coefficients (exact rational arithmetic)
# ----------------------------------------------------------------------------


def double_factorial(n):
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


def beta_opt(p):
    """Optimal beta of Eq. 21: 1 + (-1)^(p+1) (2p+2)!! / (2p+1)!!."""
    return 1 + (-1) ** (p + 1) * Fraction(double_factorial(2 * p + 2), double_factorial(2 * p + 1))


def even_pascal_matrix(size):
    """Eq. 8: the even columns of the upper-triangular Pascal matrix, A[n][m] = C(2m, n)."""
    return [[Fraction(comb(2 * m, n)) for m in range(size)] for n in range(size)]


def _solve_exact(A, b):
    """Gauss-Jordan elimination over the rationals (A square, list of lists)."""
    n = len(A)
    M = [list(row) + [b[i]] for i, row in enumerate(A)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        pv = M[col][col]
        M[col] = [x / pv for x in M[col]]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col]
                M[r] = [x - f * y for x, y in zip(M[r], M[col])]
    return [M[r][n] for r in range(n)]


def quadrature_weights(p, beta=None):
    """Weights c_n with  Delta/dt = sum_n c_n F^+-_n.

    Velocity (``beta is None``), Eq. 6: Delta v / dt = sum_{k=0..p} F_2k/(2k+1),
    n = 0..p.  Position, Eq. 7: one more even term, beta F_{2p+2}/(2p+3),
    n = 0..p+1.  The even terms follow from Eq. 8, F^+- = A F_even, so with
    row vector q of the quadrature weights, c = q A^-1, i.e. A^T c = q.
    """
    size = p + 1 if beta is None else p + 2
    q = [Fraction(1, 2 * k + 1) for k in range(p + 1)]
    if beta is not None:
        q.append(Fraction(beta) / (2 * p + 3))
    A = even_pascal_matrix(size)
    At = [[A[r][c] for r in range(size)] for c in range(size)]
    return _solve_exact(At, q)


def endpoint_coefficients(p, beta=None):
    """The same corrector written on endpoint values:
        Delta = sum_n e_n (f1^(n) +- f0^(n)) dt^(n+1),
    where F^+-_n = 1/2 h^n/n! (f1^(n) +- f0^(n)) and h = dt/2 (Eq. 1, Eq. 5), so
    e_n = c_n / (2^(n+1) n!).  Sign + for even n, - for odd n.
    """
    c = quadrature_weights(p, beta)
    return [cn / (2 ** (n + 1) * factorial(n)) for n, cn in enumerate(c)]


CORRECTORS = ("modified", "beta1", "shifted")


def corrector_beta(p, corrector="modified"):
    """beta for the position corrector variants.

    modified : beta_opt of Eq. 21 (Eq. 22-24).
    beta1    : beta = 1, the position formula exact to one order higher
               (the standard time-symmetric Hermite corrector at 4th order).
    shifted  : 2 - beta_opt; this equals the position corrector that omits the
               F_{2p+2} column of Eq. 8 altogether (the same-order velocity
               formula applied to x), which is how we read the unmodified
               6th/8th-order correctors the paper compares against.
    """
    b = beta_opt(p)
    if corrector == "modified":
        return b
    if corrector == "beta1":
        return Fraction(1)
    if corrector == "shifted":
        return 2 - b
    raise ValueError(corrector)


# ----------------------------------------------------------------------------
# Pair derivatives and potential (C part)
# ----------------------------------------------------------------------------

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_pair_derivs.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_int32, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_int64, ip, dp, dp, dp]
        lib.oracle_pair_derivs.restype = ctypes.c_int
        lib.oracle_potential.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int64, ip, dp]
        lib.oracle_potential.restype = ctypes.c_int
        lib.oracle_max_pair_rate.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_double, ctypes.c_double, dp]
        lib.oracle_max_pair_rate.restype = ctypes.c_int
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads():
    return _load().oracle_num_threads()


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class NonFiniteError(FloatingPointError):
    pass


def pair_derivs(mass, path, K=None, G=1.0, eps2=0.0, i_list=None, with_mag=False, with_scale=False):
    """a^(0..K) on each target particle from the softened pair force.

    mass : [n];  path : sequence of K+1 arrays [3][n] = x^(0..K) (x, v, a, ...)
    Returns out [K+1][3][n_i]; with ``with_mag`` also mag [K+1][n_i], the sum
    over j of the Euclidean norm of each pair term; with ``with_scale`` also
    nat [K+1][n_i], the sum over j of each pair's natural k-th derivative
    scale G m_j s^-2 omega^k (s the softened distance, omega the fastest rate
    (|x^(k)_j - x^(k)_i| / s)^(1/k) of the relative path): the size of the
    change a relative rounding of the path inputs makes in a^(k).
    """
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = mass.shape[0]
    if K is None:
        K = len(path) - 1
    P = np.ascontiguousarray(np.stack([np.asarray(path[k], dtype=np.float64).reshape(3, n)
                                       for k in range(K + 1)]))
    if i_list is None:
        n_i, ip = n, None
    else:
        il = np.ascontiguousarray(i_list, dtype=np.int64)
        n_i, ip = il.shape[0], il.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    out = np.zeros((K + 1, 3, n_i))
    mag = np.zeros((K + 1, n_i)) if with_mag else None
    nat = np.zeros((K + 1, n_i)) if with_scale else None
    rc = _load().oracle_pair_derivs(n, _dptr(mass), _dptr(P), K, float(G), float(eps2), n_i, ip,
                                    _dptr(out), _dptr(mag) if with_mag else None,
                                    _dptr(nat) if with_scale else None)
    if rc == -2:
        raise NonFiniteError("non-finite pair derivative (coincident particles with eps = 0?)")
    if rc != 0:
        raise ValueError("oracle_pair_derivs: bad arguments (%d)" % rc)
    res = (out,)
    if with_mag:
        res += (mag,)
    if with_scale:
        res += (nat,)
    return res if len(res) > 1 else out


def potential_per_particle(mass, x, G=1.0, eps2=0.0, i_list=None):
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = mass.shape[0]
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(3, n))
    if i_list is None:
        n_i, ip = n, None
    else:
        il = np.ascontiguousarray(i_list, dtype=np.int64)
        n_i, ip = il.shape[0], il.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    phi = np.zeros(n_i)
    rc = _load().oracle_potential(n, _dptr(mass), _dptr(x), float(G), float(eps2), n_i, ip, _dptr(phi))
    if rc == -2:
        raise NonFiniteError("non-finite potential")
    if rc != 0:
        raise ValueError("oracle_potential: bad arguments (%d)" % rc)
    return phi


def step_criterion(mass, x, eta, G=1.0, eps2=0.0):
    """Eq. 25: H = eta min_{i != j} ((r_ij^2 + eps^2)^(3/2) / (G (m_i + m_j)))^(1/2)
    (the minimum two-body Keplerian period scale; G = 1 in the paper)."""
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = mass.shape[0]
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(3, n))
    q = ctypes.c_double()
    rc = _load().oracle_max_pair_rate(n, _dptr(mass), _dptr(x), float(G), float(eps2), ctypes.byref(q))
    if rc != 0:
        raise ValueError("oracle_max_pair_rate: bad arguments")
    if q.value <= 0.0:
        raise ValueError("step criterion needs at least two bodies")
    return eta / np.sqrt(q.value)


def energy(mass, x, v, G=1.0, eps2=0.0):
    """E = sum 1/2 m v^2 - sum_{i<j} G m_i m_j (r_ij^2 + eps^2)^(-1/2)."""
    mass = np.asarray(mass, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64).reshape(3, -1)
    kin = 0.5 * float(np.sum(mass * np.sum(v * v, axis=0)))
    pot = 0.5 * float(np.sum(mass * potential_per_particle(mass, x, G, eps2)))
    return kin + pot


def kepler_elements(mass, x, v, k, c=0, G=1.0):
    """Osculating eccentricity vector, |e| and argument of periapsis of body k
    relative to body c, with mu = G (m_c + m_k).

    Eccentricity vector: the Laplace-Runge-Lenz vector divided by mu (Appendix A,
    first equation): e = ((|v|^2 - mu/|r|) r - (r.v) v) / mu.
    omega: angle of e measured in the orbital plane from the ascending node;
    for an orbit in the xy-plane (no node) it is atan2(e_y, e_x) taken in the
    sense of the orbital motion.
    """
    x = np.asarray(x, dtype=np.float64).reshape(3, -1)
    v = np.asarray(v, dtype=np.float64).reshape(3, -1)
    mu = G * (mass[c] + mass[k])
    r = x[:, k] - x[:, c]
    u = v[:, k] - v[:, c]
    rn = np.sqrt(r @ r)
    e = ((u @ u - mu / rn) * r - (r @ u) * u) / mu
    h = np.cross(r, u)
    node = np.array([-h[1], h[0], 0.0])
    nn = np.sqrt(node @ node)
    if nn <= 1e-14 * np.sqrt(h @ h):
        om = np.arctan2(e[1], e[0])
        if h[2] < 0:
            om = -om
    else:
        hn = h / np.sqrt(h @ h)
        nhat = node / nn
        om = np.arctan2(np.cross(nhat, e) @ hn, nhat @ e)
    return e, float(np.sqrt(e @ e)), float(om)


def wrap_angle(d):
    """Wrap an angle difference into (-pi, pi]."""
    return float(-((-d + np.pi) % (2 * np.pi) - np.pi))


# ----------------------------------------------------------------------------
# Integrator
# ----------------------------------------------------------------------------


class State:
    """Particle state of an order-2(p+1) integrator: t, m, x, v and a^(0..2p-1)."""

    def __init__(self, mass, x, v, p, derivs=None, t=0.0):
        self.mass = np.array(mass, dtype=np.float64)
        n = self.mass.shape[0]
        self.x = np.array(x, dtype=np.float64).reshape(3, n)
        self.v = np.array(v, dtype=np.float64).reshape(3, n)
        self.p = p
        self.derivs = None if derivs is None else [np.array(d, dtype=np.float64).reshape(3, n) for d in derivs]
        self.t = float(t)
        # compensation terms of x, v and t (reading R22; zero until used)
        self.cx = np.zeros((3, n))
        self.cv = np.zeros((3, n))
        self.tc = 0.0

    @property
    def n(self):
        return self.mass.shape[0]

    def copy(self):
        c = State(self.mass, self.x, self.v, self.p,
                  None if self.derivs is None else [d.copy() for d in self.derivs], self.t)
        c.cx, c.cv, c.tc = self.cx.copy(), self.cv.copy(), self.tc
        return c


def init_derivs(st, G=1.0, eps2=0.0):
    """Explicit a^(0..2p-1) at t0 (Sec. 3, second paragraph).

    Pass 1: path (x, v)            -> a, adot
    Pass 2: path (x, v, a, adot)   -> a^(2), a^(3)          (6th, 8th order)
    Pass 3: path (x, ..., a^(3))   -> a^(4), a^(5)          (8th order)
    """
    p = st.p
    need = 2 * p
    path = [st.x, st.v]
    derivs = []
    while len(derivs) < need:
        K = min(len(path) - 1, 5)    # a^(k) needs the path derivatives x^(0..k)
        out = pair_derivs(st.mass, path, K=K, G=G, eps2=eps2)
        derivs = [out[k] for k in range(K + 1)]
        path = [st.x, st.v] + derivs
    st.derivs = derivs[:need]
    return st


def predict(p, dt, x, v, derivs):
    """Taylor predictor (Sec. 3, second paragraph) with every stored a^(k).

    With x^(0) = x, x^(1) = v, x^(k+2) = a^(k) for k = 0..2p-1:
      xp = sum_{k=0..2p+1} x^(k) dt^k / k!
      vp = sum_{k=0..2p}   x^(k+1) dt^k / k!
      ap = sum_{k=0..2p-1} a^(k) dt^k / k!          (p >= 2)
      jp = sum_{k=0..2p-2} a^(k+1) dt^k / k!        (p >= 3)
    Returns the path list (xp, vp[, ap[, jp]]) that the evaluation needs
    (x^(0..p)).
    """
    xs = [x, v] + list(derivs)
    xp = sum(xs[k] * (dt ** k / factorial(k)) for k in range(2 * p + 2))
    vp = sum(xs[k + 1] * (dt ** k / factorial(k)) for k in range(2 * p + 1))
    path = [xp, vp]
    if p >= 2:
        path.append(sum(derivs[k] * (dt ** k / factorial(k)) for k in range(2 * p)))
    if p >= 3:
        path.append(sum(derivs[k + 1] * (dt ** k / factorial(k)) for k in range(2 * p - 1)))
    return path


def kahan_add(s, c, y):
    """Compensated summation (Kahan 1965), the Sec. 3.2 option: add y to a
    running sum s whose lost low-order part is c; returns the new (s, c)."""
    yc = y - c
    t = s + yc
    return t, (t - s) - yc


def correct(p, dt, x0, v0, a0, a1, corrector="modified", comp=None):
    """Modified Hermite corrector, Eq. 4-8 (Eq. 22-24 for p = 1, 2, 3).

    a0, a1 : lists a^(0..p) at the start (0) and end (1) of the step.
    F^+-_n = 1/2 h^n/n! (f^(n)(t+h) +- f^(n)(t-h)), h = dt/2, + for even n and
    - for odd n (the rows of Eq. 8).  Velocity first (f = a, Eq. 6), then
    position (f = v, f^(n) = a^(n-1), Eq. 7) using the new v1.
    comp = (cx, cv): the increments are added by compensated summation
    (reading R22) and the new (cx, cv) is returned as a third value.
    """
    h = 0.5 * dt
    cv = [float(c) for c in quadrature_weights(p)]
    cx = [float(c) for c in quadrature_weights(p, corrector_beta(p, corrector))]

    def fpm(n, f1, f0):
        s = 1.0 if n % 2 == 0 else -1.0
        return 0.5 * (h ** n / factorial(n)) * (f1 + s * f0)

    dv = sum(cv[n] * fpm(n, a1[n], a0[n]) for n in range(p + 1)) * dt
    if comp is None:
        v1 = v0 + dv
    else:
        v1, cv1 = kahan_add(v0, comp[1], dv)
    f1 = [v1] + list(a1[: p + 1])
    f0 = [v0] + list(a0[: p + 1])
    dx = sum(cx[n] * fpm(n, f1[n], f0[n]) for n in range(p + 2)) * dt
    if comp is None:
        return x0 + dx, v1
    x1, cx1 = kahan_add(x0, comp[0], dx)
    return x1, v1, (cx1, cv1)


def interpolate_higher(p, dt, a0, a1):
    """a^(p+1..2p-1) at the end of the step (reading R2).

    The degree-(2p+1) polynomial P(s), s = (t - t1)/dt, with
    d^nP/ds^n = dt^n a1^(n) at s = 0 and dt^n a0^(n) at s = -1 for n = 0..p;
    a^(k)(t1) = k! [s^k]P / dt^k.  Solved numerically with numpy.
    """
    if p < 2:
        return []
    deg = 2 * p + 1
    # Unknown coefficients d_q, q = p+1..deg; the lower ones are fixed at s = 0.
    unknown = list(range(p + 1, deg + 1))
    M = np.zeros((p + 1, len(unknown)))
    for n in range(p + 1):
        for col, q in enumerate(unknown):
            # n-th derivative of s^q at s = -1: q!/(q-n)! (-1)^(q-n)
            M[n, col] = factorial(q) / factorial(q - n) * (-1.0) ** (q - n)
    shape = np.asarray(a0[0]).shape
    rhs = np.zeros((p + 1, int(np.prod(shape))))
    for n in range(p + 1):
        known = np.zeros(int(np.prod(shape)))
        for q in range(n, p + 1):
            d_q = (dt ** q) * np.asarray(a1[q]).reshape(-1) / factorial(q)
            known = known + d_q * (factorial(q) / factorial(q - n) * (-1.0) ** (q - n))
        rhs[n] = (dt ** n) * np.asarray(a0[n]).reshape(-1) - known
    d = np.linalg.solve(M, rhs)
    out = []
    for k in range(p + 1, 2 * p):
        out.append((factorial(k) * d[k - (p + 1)] / dt ** k).reshape(shape))
    return out


def step(st, dt, n_iter, corrector="modified", G=1.0, eps2=0.0, return_iterates=False, compensated=False):
    """One P(EC)^n step (Sec. 2 end, Sec. 3) of the order-2(p+1) scheme.

    P : Taylor prediction from the t0 state.
    n times:  E : a1^(0..p) at the current iterate (reading R3 for its a, adot)
              C : v1, x1 from the t0 state and a0, a1 (Eq. 22-24).
    Then a^(p+1..2p-1)(t1) from the interpolant (R2) and the state moves to t1.
    compensated: x, v and t take their increments by compensated summation
    (reading R22); every iterate uses the carried compensation, the last one
    also updates it.
    """
    if n_iter < 1:
        raise ValueError("n_iter must be >= 1")
    p = st.p
    a0 = st.derivs[: p + 1]
    path = predict(p, dt, st.x, st.v, st.derivs)
    iterates = []
    comp = (st.cx, st.cv) if compensated else None
    for _ in range(n_iter):
        out = pair_derivs(st.mass, path, K=p, G=G, eps2=eps2)
        a1 = [out[k] for k in range(p + 1)]
        res = correct(p, dt, st.x, st.v, a0, a1, corrector, comp)
        x1, v1 = res[0], res[1]
        path = [x1, v1] + a1[: p - 1]
        iterates.append((x1, v1, a1))
    _finish(st, p, dt, a0, a1, x1, v1, res[2] if compensated else None)
    return iterates if return_iterates else st


def _finish(st, p, dt, a0, a1, x1, v1, newcomp):
    higher = interpolate_higher(p, dt, a0, a1)
    st.x, st.v = x1, v1
    st.derivs = list(a1) + higher
    if newcomp is None:
        st.t += dt
    else:
        st.cx, st.cv = newcomp
        st.t, st.tc = kahan_add(st.t, st.tc, dt)


def shift_iterate(p, d, x1, v1, a1):
    """The path x^(0..p) at t1 + d from the iterate at t1 (reading R21).

    The iterate's own Taylor series about t1, with x^(0) = x1, x^(1) = v1 and
    x^(k+2) = a1^(k) for k = 0..p:  path_f = sum_k x^(f+k) d^k / k!.  With
    d = 0 it is (x1, v1, a1, adot1) as reading R3 takes it."""
    xs = [x1, v1] + list(a1[: p + 1])
    return [sum(xs[f + k] * (d ** k / factorial(k)) for k in range(len(xs) - f)) for f in range(p + 1)]


def step_symmetric(st, eta, n_iter, corrector="modified", G=1.0, eps2=0.0, direction=1.0, compensated=False):
    """One P(EC)^n step with the implicit time-symmetric step of Sec. 3.3
    (reading R21): dt = (H_- + H_+)/2 with H (Eq. 25) at the start and at
    the end of the step.

    H_- = H(x0).  The Taylor prediction for dt = H_- gives a first end point
    and H_+ there, hence dt_1 = (H_- + H_+)/2, and the prediction is redone
    for dt_1.  Iteration k evaluates a1 at its path, which lies at t0 + dt_k,
    and corrects with that same dt_k, so that every correction takes a1 at
    the end of the step it makes (the end values of Eq. 4-8).  Before the
    next iteration, H_+ at this evaluation point gives dt_(k+1), and the new
    iterate is moved to t0 + dt_(k+1) along its own Taylor series.  The step
    taken is the last correction's dt.  ``direction`` = -1 integrates
    backwards.  Returns that dt."""
    if n_iter < 1:
        raise ValueError("n_iter must be >= 1")
    p = st.p
    a0 = st.derivs[: p + 1]
    Hm = step_criterion(st.mass, st.x, eta, G, eps2)
    path = predict(p, direction * Hm, st.x, st.v, st.derivs)
    dt = direction * 0.5 * (Hm + step_criterion(st.mass, path[0], eta, G, eps2))
    path = predict(p, dt, st.x, st.v, st.derivs)
    comp = (st.cx, st.cv) if compensated else None
    for k in range(n_iter):
        out = pair_derivs(st.mass, path, K=p, G=G, eps2=eps2)
        a1 = [out[j] for j in range(p + 1)]
        res = correct(p, dt, st.x, st.v, a0, a1, corrector, comp)
        x1, v1 = res[0], res[1]
        if k + 1 < n_iter:
            dt_next = direction * 0.5 * (Hm + step_criterion(st.mass, path[0], eta, G, eps2))
            path = shift_iterate(p, dt_next - dt, x1, v1, a1)
            dt = dt_next
    _finish(st, p, dt, a0, a1, x1, v1, res[2] if compensated else None)
    return dt


def run(st, dt, n_steps, n_iter, corrector="modified", G=1.0, eps2=0.0, callback=None):
    for s in range(n_steps):
        step(st, dt, n_iter, corrector, G, eps2)
        if callback is not None:
            callback(s, st)
    return st
