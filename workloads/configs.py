"""The five synthetic workloads (seeded).

Every generator returns a dict with ``mass`` [n], ``x`` [3][n], ``v`` [3][n]
(FP64, barycentric frame, G = 1) and the run parameters of the workload.
Seeds: ``numpy.random.Generator(PCG64(1000 + index))``; the batched workload
draws system s from ``SeedSequence(1003).spawn(n_systems)[s]``.
"""
import numpy as np

from .orbits import elements_to_cartesian, to_barycentric

TWO_PI = 2.0 * np.pi


def _rng(index):
    return np.random.Generator(np.random.PCG64(1000 + index))


def _disc(rng, n_tot, m_central, m_body, a, e_sigma, i_sigma):
    n = n_tot - 1
    e = rng.rayleigh(e_sigma, n)
    e = np.minimum(e, 0.95)
    inc = rng.rayleigh(i_sigma, n)
    node, peri, mean = (rng.uniform(0.0, TWO_PI, n) for _ in range(3))
    r, v = elements_to_cartesian(m_central + m_body, a, e, inc, node, peri, mean)
    mass = np.concatenate([[m_central], np.full(n, m_body)])
    x = np.concatenate([np.zeros((3, 1)), r], axis=1)
    vv = np.concatenate([np.zeros((3, 1)), v], axis=1)
    x, vv = to_barycentric(mass, x, vv)
    return mass, np.ascontiguousarray(x), np.ascontiguousarray(vv)


def kepler_two_body(e=0.5, a=1.0, m_central=1.0, m=1e-3, mean_anomaly=0.0):
    """Two-body orbit in the xy-plane, starting at periapsis by default."""
    r, v = elements_to_cartesian(m_central + m, a, e, 0.0, 0.0, 0.0, mean_anomaly)
    mass = np.array([m_central, m])
    x = np.concatenate([np.zeros((3, 1)), r.reshape(3, 1)], axis=1)
    vv = np.concatenate([np.zeros((3, 1)), v.reshape(3, 1)], axis=1)
    x, vv = to_barycentric(mass, x, vv)
    period = TWO_PI * np.sqrt(a ** 3 / (m_central + m))
    return dict(name="kepler_two_body", mass=mass, x=x, v=vv, period=period, G=1.0, eps2=0.0)


def ring64(n=64):
    """Central mass 1 plus 63 planetesimals of 1e-9 near a = 1 (4th order, n = 2)."""
    rng = _rng(0)
    a = rng.uniform(0.9, 1.1, n - 1)
    mass, x, v = _disc(rng, n, 1.0, 1e-9, a, 0.01, 0.005)
    return dict(name="ring64", mass=mass, x=x, v=v, order=4, n_iter=2, dt=TWO_PI / 1000,
                steps=10000, G=1.0, eps2=0.0)


def disc16k(n=16384):
    """Stellar disc around a central mass 1.0: 16383 stars of 1e-7, a log-uniform in
    [0.1, 1], e ~ Rayleigh(0.05), i ~ Rayleigh(0.02) (8th order, n = 3)."""
    rng = _rng(1)
    a = np.exp(rng.uniform(np.log(0.1), np.log(1.0), n - 1))
    mass, x, v = _disc(rng, n, 1.0, 1e-7, a, 0.05, 0.02)
    return dict(name="disc16k", mass=mass, x=x, v=v, order=8, n_iter=3, dt=TWO_PI / 2000,
                steps=100, G=1.0, eps2=0.0)


def plummer_cluster(n_stars=131072, m_bh=0.01):
    """Equal-mass Plummer sphere (total mass 1, virial radius 1, so the scale
    radius is 3 pi / 16) plus a central mass 0.01 at rest at the origin.
    Radii by the inverse cumulative mass with X ~ U(0, 0.999] (the outer 0.1 %
    of the mass is cut); speeds q v_esc(r) with q drawn by rejection on
    q^2 (1 - q^2)^(7/2); isotropic directions (6th order, n = 2, eps = 1e-4)."""
    rng = _rng(2)
    ap = 3.0 * np.pi / 16.0
    X = 0.999 * (1.0 - rng.random(n_stars))            # (0, 0.999]
    r = ap / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    def iso(k):
        cz = rng.uniform(-1.0, 1.0, k)
        ph = rng.uniform(0.0, TWO_PI, k)
        s = np.sqrt(1.0 - cz * cz)
        return np.stack([s * np.cos(ph), s * np.sin(ph), cz])
    pos = iso(n_stars) * r
    q = np.empty(n_stars)
    todo = np.arange(n_stars)
    while todo.size:
        qq = rng.random(todo.size)
        yy = 0.1 * rng.random(todo.size)
        ok = yy < qq * qq * (1.0 - qq * qq) ** 3.5
        q[todo[ok]] = qq[ok]
        todo = todo[~ok]
    vesc = np.sqrt(2.0) * (r * r + ap * ap) ** (-0.25)
    vel = iso(n_stars) * (q * vesc)
    mass = np.concatenate([np.full(n_stars, 1.0 / n_stars), [m_bh]])
    x = np.concatenate([pos, np.zeros((3, 1))], axis=1)
    v = np.concatenate([vel, np.zeros((3, 1))], axis=1)
    x, v = to_barycentric(mass, x, v)
    return dict(name="plummer_cluster", mass=mass, x=np.ascontiguousarray(x), v=np.ascontiguousarray(v),
                order=6, n_iter=2, dt=1.0 / 4096, steps=10, G=1.0, eps2=1e-8)


def _hill_log_gaps(m_planets, m_star, delta):
    h = ((m_planets[:-1] + m_planets[1:]) / (3.0 * m_star)) ** (1.0 / 3.0)
    x = 0.5 * delta * h
    if np.any(x >= 1.0):
        return None
    return np.log((1.0 + x) / (1.0 - x))


def _one_system(rng, n):
    m_star = 1.0
    k = n - 1
    mp = np.exp(rng.uniform(np.log(1e-7), np.log(1e-3), k))
    L = np.log(5.0 / 0.05)
    delta = 8.0
    gaps = _hill_log_gaps(mp, m_star, delta)
    if gaps is None or gaps.sum() > L:
        lo, hi = 0.0, 8.0
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            g = _hill_log_gaps(mp, m_star, mid)
            if g is not None and g.sum() <= L:
                lo = mid
            else:
                hi = mid
        delta = lo
        gaps = _hill_log_gaps(mp, m_star, delta)
    spare = L - gaps.sum()
    extra = rng.dirichlet(np.ones(k + 1)) * spare
    loga = np.log(0.05) + np.concatenate([[0.0], np.cumsum(gaps)]) + np.cumsum(extra[:k])
    a = np.exp(loga)
    e = np.minimum(rng.rayleigh(0.02, k), 0.9)
    inc = rng.rayleigh(0.01, k)
    node, peri, mean = (rng.uniform(0.0, TWO_PI, k) for _ in range(3))
    r, v = elements_to_cartesian(m_star + mp, a, e, inc, node, peri, mean)
    mass = np.concatenate([[m_star], mp])
    x = np.concatenate([np.zeros((3, 1)), r], axis=1)
    vv = np.concatenate([np.zeros((3, 1)), v], axis=1)
    x, vv = to_barycentric(mass, x, vv)
    p_inner = TWO_PI * np.sqrt(a[0] ** 3 / (m_star + mp[0]))
    return mass, x, vv, p_inner / 500.0, delta


def batch_systems(n_systems=4096, n_min=3, n_max=64):
    """Independent planetary systems: a star of 1.0 plus N-1 planets, N ~ U{3..64},
    planet masses log-uniform in [1e-7, 1e-3], a in [0.05, 5] with mutual Hill
    spacing of at most 8 (the largest spacing <= 8 that fits the range),
    e ~ Rayleigh(0.02), i ~ Rayleigh(0.01); per-system dt = P_inner / 500
    (8th order, n = 3, 1000 steps).

    Returns concatenated SoA arrays with ``offsets`` [n_systems + 1]."""
    seqs = np.random.SeedSequence(1003).spawn(n_systems)
    sizes = np.random.Generator(np.random.PCG64(1003)).integers(n_min, n_max + 1, n_systems)
    ms, xs, vs, dts, deltas = [], [], [], [], []
    for s in range(n_systems):
        rng = np.random.Generator(np.random.PCG64(seqs[s]))
        m, x, v, dt, d = _one_system(rng, int(sizes[s]))
        ms.append(m); xs.append(x); vs.append(v); dts.append(dt); deltas.append(d)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return dict(name="batch_systems", mass=np.concatenate(ms), x=np.ascontiguousarray(np.concatenate(xs, axis=1)),
                v=np.ascontiguousarray(np.concatenate(vs, axis=1)), offsets=offsets, dt=np.array(dts),
                hill_spacing=np.array(deltas), order=8, n_iter=3, steps=1000, G=1.0, eps2=0.0)


def large_disc(n=1048576):
    """Central mass 1.0 plus stars of 1e-9 with surface density ~ r^-1.5 on
    [0.05, 1] (so M(<r) ~ r^0.5: a = (sqrt(0.05) + U (1 - sqrt(0.05)))^2),
    e ~ Rayleigh(0.1), i ~ Rayleigh(0.05) (8th order, n = 3)."""
    rng = _rng(4)
    u = rng.random(n - 1)
    a = (np.sqrt(0.05) + u * (1.0 - np.sqrt(0.05))) ** 2
    mass, x, v = _disc(rng, n, 1.0, 1e-9, a, 0.1, 0.05)
    return dict(name="large_disc", mass=mass, x=x, v=v, order=8, n_iter=3, dt=TWO_PI / 2000,
                steps=1, G=1.0, eps2=0.0)


def disc100(n_bodies=100, realization=0):
    """The paper's N-body test (Sec. 3.3, Table 1): 100 bodies of 1e-5 around a
    central mass 1, semi-major axes evenly log-spaced in [0.1, 10], e ~
    Rayleigh(0.06) and i ~ Rayleigh(0.12) (sigma_i = 2 sigma_e = 0.12), angles
    uniform; eps = 1e-6, t_end = 100 pi.  Seeded: no seed is given.
    realization k > 0 draws the same recipe from another seed (the paper's
    figures come from one unknown draw)."""
    rng = _rng(5) if realization == 0 else _rng(100000 + int(realization))
    a = np.geomspace(0.1, 10.0, n_bodies)
    mass, x, v = _disc(rng, n_bodies + 1, 1.0, 1e-5, a, 0.06, 0.12)
    return dict(name="disc100", mass=mass, x=x, v=v, order=8, eps2=1e-12, t_end=100 * np.pi, G=1.0)


CONFIGS = {
    "ring64": ring64,
    "disc16k": disc16k,
    "plummer_cluster": plummer_cluster,
    "batch_systems": batch_systems,
    "large_disc": large_disc,
    "disc100": disc100,
}
