"""Pins of the oracle's integrator (predictor, corrector, interpolation, P(EC)^n,
initialisation) against what the paper and the mathematics fix:

* exactness of the Taylor predictor and of the Hermite interpolant on
  polynomials of the degree they are built for;
* initial derivatives against 30-digit derivatives of the exact two-body
  (Kepler) solution;
* convergence order 2(p+1) as dt halves (Sec. 2: order 2(p+1));
* time symmetry of the iterated scheme (Sec. 2.1 end: time symmetric when
  iterated to convergence);
* Sec. 3.1 claims: no secular energy error; the modified corrector's
  periapsis drift is far below the unmodified ones; about three orders of
  magnitude less energy error from 4th to 6th order at dt = 2^-4; n = 2 far
  better than n = 1, n = 3 close to n = 4 (Fig. 4 discussion);
* Eq. 21 recovered physically: the beta at which the periapsis drift
  vanishes, fitted from two unmodified runs, is beta_opt;
* momentum conservation and bitwise checkpoint/resume.
"""
from math import factorial

import mpmath
import numpy as np
import pytest

from oracle import hermite_oracle as ho
from workloads import kepler_two_body, ring64

EPS2_2BODY = 1e-16      # eps = 1e-8 for the paper's 2-body tests (Sec. 3)


def _poly(rng, deg, shape=(3, 4)):
    return [rng.normal(size=shape) / factorial(k) for k in range(deg + 1)]


def _pd(c, n, t):
    return sum(c[k] * (factorial(k) / factorial(k - n)) * t ** (k - n) for k in range(n, len(c)))


@pytest.mark.parametrize("p", [1, 2, 3])
def test_predictor_exact_on_polynomials(p):
    rng = np.random.default_rng(p)
    c = _poly(rng, 2 * p + 1)
    t0, dt = 0.4, 0.3
    derivs = [_pd(c, k + 2, t0) for k in range(2 * p)]
    path = ho.predict(p, dt, _pd(c, 0, t0), _pd(c, 1, t0), derivs)
    assert len(path) == p + 1
    for k, q in enumerate(path):
        assert np.allclose(q, _pd(c, k, t0 + dt), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("p", [2, 3])
def test_interpolation_exact_on_polynomials(p):
    rng = np.random.default_rng(40 + p)
    c = _poly(rng, 2 * p + 1)            # a(t) of degree 2p+1
    t0, dt = -0.1, 0.35
    t1 = t0 + dt
    a0 = [_pd(c, k, t0) for k in range(p + 1)]
    a1 = [_pd(c, k, t1) for k in range(p + 1)]
    hi = ho.interpolate_higher(p, dt, a0, a1)
    assert len(hi) == p - 1
    for j, k in enumerate(range(p + 1, 2 * p)):
        ref = _pd(c, k, t1)
        assert np.allclose(hi[j], ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_interpolation_none_at_4th_order():
    assert ho.interpolate_higher(1, 0.1, [np.zeros(3)] * 2, [np.zeros(3)] * 2) == []


def _kepler_exact_derivs(e, a, M, m, nder, t=0.0):
    """Derivatives 0..nder of the planet's barycentric position on the exact
    Kepler orbit starting at periapsis (30 digits, mpmath)."""
    mpmath.mp.dps = 30
    mu = mpmath.mpf(M + m)
    a_ = mpmath.mpf(a)
    e_ = mpmath.mpf(e)
    nmot = mpmath.sqrt(mu / a_ ** 3)
    fac = mpmath.mpf(M) / mu

    def ecc_anom(tt):
        Mn = nmot * tt
        E = Mn
        for _ in range(80):
            E = E - (E - e_ * mpmath.sin(E) - Mn) / (1 - e_ * mpmath.cos(E))
        return E

    def comp(c):
        def f(tt):
            E = ecc_anom(tt)
            if c == 0:
                return fac * a_ * (mpmath.cos(E) - e_)
            return fac * a_ * mpmath.sqrt(1 - e_ * e_) * mpmath.sin(E)
        return f
    return [[float(v) for v in mpmath.diffs(comp(c), t, nder)] for c in (0, 1)]


@pytest.mark.parametrize("p", [1, 2, 3])
def test_init_derivs_match_exact_kepler(p):
    e, a, M, m = 0.5, 1.0, 1.0, 1e-3
    w = kepler_two_body(e=e, a=a, m_central=M, m=m)
    st = ho.State(w["mass"], w["x"], w["v"], p)
    ho.init_derivs(st)
    assert len(st.derivs) == 2 * p
    ref = _kepler_exact_derivs(e, a, M, m, 2 * p + 1)
    for k in range(2 * p):
        for c in (0, 1):
            exp = ref[c][k + 2]
            got = st.derivs[k][c, 1]
            scale = max(abs(ref[0][k + 2]), abs(ref[1][k + 2]))
            assert abs(got - exp) <= 1e-11 * scale, (k, c, got, exp)


def _kepler_run(order, n_iter, steps, dt, e=0.5, corrector="modified", eps2=0.0, track_energy=False):
    w = kepler_two_body(e=e)
    p = order // 2 - 1
    st = ho.State(w["mass"], w["x"], w["v"], p)
    ho.init_derivs(st, eps2=eps2)
    x0 = st.x.copy()
    E0 = ho.energy(st.mass, st.x, st.v, eps2=eps2)
    _, _, om0 = ho.kepler_elements(st.mass, st.x, st.v, 1)
    dE = []
    for _ in range(steps):
        ho.step(st, dt, n_iter, corrector, eps2=eps2)
        if track_energy:
            dE.append(abs(ho.energy(st.mass, st.x, st.v, eps2=eps2) / E0 - 1.0))
    _, _, om = ho.kepler_elements(st.mass, st.x, st.v, 1)
    return dict(st=st, x0=x0, dE=np.array(dE), dom=ho.wrap_angle(om - om0), period=w["period"])


@pytest.mark.parametrize("order,nper", [(4, 128), (6, 64), (8, 48)])
def test_convergence_order(order, nper):
    # After exactly one period the exact relative orbit is back at its start.
    errs = []
    for k in (nper, 2 * nper):
        period = kepler_two_body(e=0.5)["period"]
        r = _kepler_run(order, 4, k, period / k)
        errs.append(np.abs(r["st"].x - r["x0"]).max())
    slope = np.log2(errs[0] / errs[1])
    assert abs(slope - order) <= 0.3, (order, errs, slope)


@pytest.mark.parametrize("order", [4, 6, 8])
def test_time_symmetry(order):
    dt = 2 * np.pi / 100
    w = kepler_two_body(e=0.5)
    p = order // 2 - 1
    st = ho.State(w["mass"], w["x"], w["v"], p)
    ho.init_derivs(st)
    x0 = st.x.copy()
    for _ in range(100):
        ho.step(st, dt, 8)
    for _ in range(100):
        ho.step(st, -dt, 8)
    assert np.abs(st.x - x0).max() < 1e-13


def test_time_symmetry_needs_iteration():
    # n = 1 (standard Hermite) is not time symmetric: the same round trip misses.
    dt = 2 * np.pi / 100
    w = kepler_two_body(e=0.5)
    st = ho.State(w["mass"], w["x"], w["v"], 1)
    ho.init_derivs(st)
    x0 = st.x.copy()
    for s in (dt, -dt):
        for _ in range(100):
            ho.step(st, s, 1)
    assert np.abs(st.x - x0).max() > 1e-5


@pytest.fixture(scope="module")
def paper_kepler_runs():
    """Sec. 3.1 set-up: a = 1, e = 0.1, planet 1e-3 around 1, dt = 2^-4, n = 3,
    eps = 1e-8; here 10 orbits instead of t = 100 pi."""
    out = {}
    for order in (4, 6, 8):
        for corr in ho.CORRECTORS:
            if order == 8 and corr == "shifted":
                continue
            steps = int(round(10 * 2 * np.pi / 2 ** -4))
            out[(order, corr)] = _kepler_run(order, 3, steps, 2 ** -4, e=0.1, corrector=corr,
                                             eps2=EPS2_2BODY, track_energy=True)
    return out


def test_periapsis_drift_modified_vs_unmodified(paper_kepler_runs):
    r = paper_kepler_runs
    for order, factor in ((4, 0.01), (6, 0.01), (8, 0.5)):
        mod = abs(r[(order, "modified")]["dom"])
        base = abs(r[(order, "beta1")]["dom"])
        assert mod < factor * base, (order, mod, base)
    for order in (4, 6):
        assert abs(r[(order, "modified")]["dom"]) < 0.01 * abs(r[(order, "shifted")]["dom"])


def test_eq21_beta_from_zero_periapsis_drift(paper_kepler_runs):
    # The leading periapsis drift is linear in beta; its zero, found from the
    # beta = 1 and beta = 2 - beta_opt runs, is Eq. 21's beta_opt.
    r = paper_kepler_runs
    for order in (4, 6):
        p = order // 2 - 1
        b1, bs = 1.0, float(ho.corrector_beta(p, "shifted"))
        d1, ds = r[(order, "beta1")]["dom"], r[(order, "shifted")]["dom"]
        beta_star = b1 - d1 * (bs - b1) / (ds - d1)
        bo = float(ho.beta_opt(p))
        assert abs(beta_star - bo) <= 0.02 * abs(bo), (order, beta_star, bo)


def test_energy_bounded_and_order_gap(paper_kepler_runs):
    r = paper_kepler_runs
    for order in (4, 6, 8):
        dE = r[(order, "modified")]["dE"]
        h = len(dE) // 2
        # no secular growth: the second half is no worse than the first (with slack)
        assert dE[h:].max() <= 1.5 * dE[:h].max() + 5e-15
    e4 = r[(4, "modified")]["dE"].max()
    e6 = r[(6, "modified")]["dE"].max()
    e8 = r[(8, "modified")]["dE"].max()
    assert e6 < 1e-3 * e4 * 5          # "about three orders of magnitude"
    assert e8 < 1e-2 * e6              # "2-3 orders smaller", round-off dominated
    assert e8 < 1e-13


def test_iteration_count_sweep():
    # Fig. 4 discussion: n = 2 radically better than n = 1 (whose energy error
    # grows secularly); n = 3 and n = 4 behave nearly identically.
    steps = int(round(10 * 2 * np.pi / 2 ** -4))
    res = {n: _kepler_run(4, n, steps, 2 ** -4, e=0.1, eps2=EPS2_2BODY, track_energy=True)["dE"]
           for n in (1, 2, 3, 4)}
    assert res[1].max() > 10 * res[2].max()
    h = len(res[1]) // 2
    assert res[1][h:].max() > 1.5 * res[1][:h].max()
    assert abs(res[3].max() - res[4].max()) < 0.05 * res[3].max()


def test_momentum_and_centre_of_mass_conserved():
    w = ring64()
    st = ho.State(w["mass"], w["x"], w["v"], 1)
    ho.init_derivs(st)
    P0 = (st.v * st.mass).sum(axis=1)
    scale = (np.abs(st.v) * st.mass).sum()
    for _ in range(20):
        ho.step(st, w["dt"], w["n_iter"])
    P1 = (st.v * st.mass).sum(axis=1)
    assert np.abs(P1 - P0).max() <= 1e-15 * scale
    for k, d in enumerate(st.derivs):
        assert np.abs((d * st.mass).sum(axis=1)).max() <= 1e-13 * (np.abs(d) * st.mass).sum()


def test_checkpoint_resume_bitwise():
    w = kepler_two_body(e=0.3)
    st = ho.State(w["mass"], w["x"], w["v"], 3)
    ho.init_derivs(st)
    a = st.copy()
    for _ in range(20):
        ho.step(a, 0.05, 3)
    b = st.copy()
    for _ in range(10):
        ho.step(b, 0.05, 3)
    b = b.copy()
    for _ in range(10):
        ho.step(b, 0.05, 3)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.v, b.v)
    assert all(np.array_equal(p, q) for p, q in zip(a.derivs, b.derivs))


def test_step_rejects_bad_iteration_count():
    w = kepler_two_body()
    st = ho.State(w["mass"], w["x"], w["v"], 1)
    ho.init_derivs(st)
    with pytest.raises(ValueError):
        ho.step(st, 0.1, 0)
