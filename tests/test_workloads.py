"""The seeded synthetic inputs follow the recipes the benchmarks and parity
tests state for them (masses, element ranges and distributions, barycentric
frame, run parameters), and they are reproducible.  The elements are
recovered here from the heliocentric two-body relations (a from the vis-viva
energy, e and i from the angular momentum), not from the generator's own
routines."""
import math

import numpy as np
import pytest

from workloads import batch_systems, disc100, disc16k, kepler_two_body, large_disc, plummer_cluster, ring64

RAYLEIGH_MEAN = math.sqrt(math.pi / 2.0)     # mean of Rayleigh(sigma) is sigma sqrt(pi / 2)


def _helio_elements(mass, x, v, c=0, idx=None):
    """a, e, i of bodies idx around body c (mu = G (m_c + m_k), G = 1)."""
    idx = np.arange(len(mass)) if idx is None else np.asarray(idx)
    idx = idx[idx != c]
    r = x[:, idx] - x[:, c:c + 1]
    u = v[:, idx] - v[:, c:c + 1]
    mu = mass[c] + mass[idx]
    rn = np.linalg.norm(r, axis=0)
    a = 1.0 / (2.0 / rn - np.sum(u * u, axis=0) / mu)
    h = np.cross(r.T, u.T).T
    hn = np.linalg.norm(h, axis=0)
    e = np.sqrt(np.maximum(0.0, 1.0 - hn * hn / (mu * a)))
    inc = np.arccos(np.clip(h[2] / hn, -1.0, 1.0))
    return a, e, inc


def _barycentric(mass, x, v):
    scale_x = np.abs(x).max() * mass.sum()
    scale_v = np.abs(v).max() * mass.sum()
    assert np.abs(x @ mass).max() <= 1e-14 * scale_x
    assert np.abs(v @ mass).max() <= 1e-14 * scale_v


def test_kepler_two_body():
    w = kepler_two_body(e=0.5)
    a, e, inc = _helio_elements(w["mass"], w["x"], w["v"])
    assert a[0] == pytest.approx(1.0, rel=1e-14) and e[0] == pytest.approx(0.5, rel=1e-13) and inc[0] == 0.0
    assert w["period"] == pytest.approx(2.0 * math.pi / math.sqrt(1.001), rel=1e-15)
    # at periapsis by default: on the +x axis at a (1 - e)
    r = w["x"][:, 1] - w["x"][:, 0]
    assert r[0] == pytest.approx(0.5, rel=1e-14) and abs(r[1]) < 1e-15
    _barycentric(w["mass"], w["x"], w["v"])


def test_ring64():
    w = ring64()
    m = w["mass"]
    assert len(m) == 64 and m[0] == 1.0 and np.all(m[1:] == 1e-9)
    a, e, inc = _helio_elements(m, w["x"], w["v"])
    assert a.min() >= 0.9 * (1 - 1e-12) and a.max() <= 1.1 * (1 + 1e-12)
    assert e.mean() == pytest.approx(0.01 * RAYLEIGH_MEAN, rel=0.3)
    assert inc.mean() == pytest.approx(0.005 * RAYLEIGH_MEAN, rel=0.3)
    assert (w["order"], w["n_iter"], w["steps"]) == (4, 2, 10000) and w["dt"] == pytest.approx(2 * math.pi / 1000)
    _barycentric(m, w["x"], w["v"])


def test_disc16k():
    w = disc16k()
    m = w["mass"]
    assert len(m) == 16384 and m[0] == 1.0 and np.all(m[1:] == 1e-7)
    a, e, inc = _helio_elements(m, w["x"], w["v"])
    assert a.min() >= 0.1 * (1 - 1e-12) and a.max() <= 1.0 * (1 + 1e-12)
    # log-uniform: log a uniform on [log 0.1, 0] (mean and spread of a uniform law)
    la = np.log(a)
    assert la.mean() == pytest.approx(0.5 * math.log(0.1), rel=0.02)
    assert la.std() == pytest.approx(abs(math.log(0.1)) / math.sqrt(12.0), rel=0.03)
    assert e.mean() == pytest.approx(0.05 * RAYLEIGH_MEAN, rel=0.03)
    assert inc.mean() == pytest.approx(0.02 * RAYLEIGH_MEAN, rel=0.03)
    assert (w["order"], w["n_iter"], w["eps2"]) == (8, 3, 0.0) and w["dt"] == pytest.approx(2 * math.pi / 2000)
    _barycentric(m, w["x"], w["v"])
    # reproducible
    w2 = disc16k()
    assert np.array_equal(w["x"], w2["x"]) and np.array_equal(w["v"], w2["v"])


def test_plummer_cluster():
    w = plummer_cluster()
    m = w["mass"]
    assert len(m) == 131073 and np.all(m[:-1] == 1.0 / 131072) and m[-1] == 0.01
    _barycentric(m, w["x"], w["v"])
    stars = slice(0, 131072)
    # radii and velocities about the central mass (drawn at rest at the origin
    # before the shift to the barycentre)
    ap = 3.0 * math.pi / 16.0
    r = np.linalg.norm(w["x"][:, stars] - w["x"][:, -1:], axis=0)
    # mass inside r for a Plummer sphere: r^3 / (r^2 + a^2)^(3/2); the cut keeps X <= 0.999
    X = r ** 3 / (r * r + ap * ap) ** 1.5
    assert X.max() <= 0.999 * (1 + 1e-9)
    assert np.median(X) == pytest.approx(0.4995, abs=0.005)
    # kinetic energy of a Plummer sphere of mass 1 and virial radius 1 is 1/4
    # (the cut outer 0.1 % and the central mass change it by well under 2 %)
    vrel = w["v"][:, stars] - w["v"][:, -1:]
    T = 0.5 * np.sum(m[stars] * np.sum(vrel * vrel, axis=0))
    assert T == pytest.approx(0.25, rel=0.02)
    # speeds below the local escape speed
    vesc = math.sqrt(2.0) * (r * r + ap * ap) ** -0.25
    assert np.all(np.linalg.norm(vrel, axis=0) < vesc)
    assert (w["order"], w["n_iter"], w["eps2"]) == (6, 2, 1e-8) and w["dt"] == 1.0 / 4096


@pytest.fixture(scope="module")
def batch():
    return batch_systems()


def test_batch_systems_sizes_and_masses(batch):
    off = batch["offsets"]
    sz = np.diff(off)
    assert len(sz) == 4096 and sz.min() >= 3 and sz.max() <= 64
    assert set(np.unique(sz)) == set(range(3, 65))          # every size drawn
    m = batch["mass"]
    stars = off[:-1]
    assert np.all(m[stars] == 1.0)
    planets = np.ones(len(m), bool)
    planets[stars] = False
    assert m[planets].min() >= 1e-7 and m[planets].max() <= 1e-3
    # log-uniform planet masses
    assert np.log10(m[planets]).mean() == pytest.approx(-5.0, abs=0.05)
    assert (batch["order"], batch["n_iter"], batch["steps"]) == (8, 3, 1000)


def test_batch_systems_orbits(batch):
    off, m, x, v = batch["offsets"], batch["mass"], batch["x"], batch["v"]
    es, incs = [], []
    rng = np.random.default_rng(0)
    for s in rng.choice(4096, 256, replace=False):
        lo, hi = off[s], off[s + 1]
        ms, xs, vs = m[lo:hi], x[:, lo:hi], v[:, lo:hi]
        _barycentric(ms, xs, vs)
        a, e, inc = _helio_elements(ms, xs, vs)
        assert a.min() >= 0.05 * (1 - 1e-9) and a.max() <= 5.0 * (1 + 1e-9), s
        # dt = P_inner / 500 with the innermost planet's period
        k = np.argmin(a)
        p_inner = 2 * math.pi * math.sqrt(a[k] ** 3 / (1.0 + ms[1:][k]))
        assert batch["dt"][s] == pytest.approx(p_inner / 500.0, rel=1e-10), s
        # neighbours at least the recorded mutual Hill spacing apart (<= 8)
        order = np.argsort(a)
        a_s, mp = a[order], ms[1:][order]
        rh = 0.5 * (a_s[:-1] + a_s[1:]) * ((mp[:-1] + mp[1:]) / 3.0) ** (1.0 / 3.0)
        d = batch["hill_spacing"][s]
        assert 0.0 < d <= 8.0
        assert np.all(np.diff(a_s) >= d * rh * (1 - 1e-6)), s
        es.append(e)
        incs.append(inc)
    es, incs = np.concatenate(es), np.concatenate(incs)
    assert es.mean() == pytest.approx(0.02 * RAYLEIGH_MEAN, rel=0.05)
    assert incs.mean() == pytest.approx(0.01 * RAYLEIGH_MEAN, rel=0.05)


def test_large_disc():
    w = large_disc()
    m = w["mass"]
    assert len(m) == 1048576 and m[0] == 1.0 and np.all(m[1:] == 1e-9)
    idx = np.arange(1, len(m), 97)                 # a sample of about 10800 stars
    a, e, inc = _helio_elements(m, w["x"], w["v"], idx=idx)
    assert a.min() >= 0.05 * (1 - 1e-12) and a.max() <= 1.0 * (1 + 1e-12)
    # surface density r^-1.5: the enclosed mass grows as sqrt(a), so sqrt(a) is uniform
    sa = np.sqrt(a)
    lo = math.sqrt(0.05)
    assert sa.mean() == pytest.approx(0.5 * (lo + 1.0), rel=0.01)
    assert sa.std() == pytest.approx((1.0 - lo) / math.sqrt(12.0), rel=0.03)
    assert e.mean() == pytest.approx(0.1 * RAYLEIGH_MEAN, rel=0.03)
    assert inc.mean() == pytest.approx(0.05 * RAYLEIGH_MEAN, rel=0.03)
    assert (w["order"], w["n_iter"], w["eps2"]) == (8, 3, 0.0)


def test_disc100_and_its_draws():
    w = disc100()
    m = w["mass"]
    assert len(m) == 101 and m[0] == 1.0 and np.all(m[1:] == 1e-5)
    a, e, inc = _helio_elements(m, w["x"], w["v"])
    # semi-major axes evenly spaced in log a on [0.1, 10], endpoints included
    assert np.allclose(a, np.geomspace(0.1, 10.0, 100), rtol=1e-11)
    assert e.mean() == pytest.approx(0.06 * RAYLEIGH_MEAN, rel=0.25)
    assert inc.mean() == pytest.approx(0.12 * RAYLEIGH_MEAN, rel=0.25)
    assert w["eps2"] == 1e-12 and w["t_end"] == pytest.approx(100 * math.pi)
    _barycentric(m, w["x"], w["v"])
    # draw 0 is the default; other draws differ, keep the recipe, and repeat
    assert np.array_equal(disc100(realization=0)["x"], w["x"])
    w3 = disc100(realization=3)
    assert not np.array_equal(w3["x"], w["x"])
    assert np.array_equal(disc100(realization=3)["v"], w3["v"])
    a3, _, _ = _helio_elements(w3["mass"], w3["x"], w3["v"])
    assert np.allclose(a3, np.geomspace(0.1, 10.0, 100), rtol=1e-11)
