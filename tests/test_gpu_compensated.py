"""GPU path with compensated summation in the time integration (Sec. 3.2,
reading R22): parity with the oracle's compensated steps (fixed and
variable), the free-particle and Kepler round-off properties on the GPU, and
checkpoint/resume of the compensation terms."""
import sys
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import hermite_oracle as ho
from paper_2006_02501_amd import Hermite, HermiteError
from parity_util import disc_path, rel_max
from workloads import disc100, kepler_two_body, ring64

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _run_pair(order, w, dt, n_iter, steps, eps2=0.0):
    p = order // 2 - 1
    o = ho.State(w["mass"], w["x"], w["v"], p)
    ho.init_derivs(o, eps2=eps2)
    n = len(w["mass"])
    h = Hermite(order, n, eps2=eps2, compensated=True, device=DEV)
    st = h.state(w["mass"], w["x"], w["v"])
    h.init(st)
    for _ in range(steps):
        ho.step(o, dt, n_iter, eps2=eps2, compensated=True)
        h.step(st, dt, n_iter)
    d = st.host()
    h.close()
    return o, d


@pytest.mark.parametrize("case", ["kepler4", "kepler8", "ring64", "disc700"])
def test_compensated_step_parity(case):
    _say("compensated step parity %s" % case)
    if case.startswith("kepler"):
        w = kepler_two_body(e=0.5)
        order, dt, n_iter = int(case[-1]), w["period"] / 200, 3
    elif case == "ring64":
        w = ring64()
        order, dt, n_iter = 4, w["dt"], w["n_iter"]
    else:
        w, _ = disc_path(700, 1)
        order, dt, n_iter = 8, 2 * np.pi / 2000, 3
    o, g = _run_pair(order, w, dt, n_iter, 1)
    assert rel_max(g["x"], o.x) <= 1e-13 and rel_max(g["v"], o.v) <= 1e-13
    o, g = _run_pair(order, w, dt, n_iter, 50)
    assert rel_max(g["x"], o.x) <= 1e-11 and rel_max(g["v"], o.v) <= 1e-11
    # t follows the same compensated rule on the host: bitwise the oracle's
    assert g["t"] == o.t and g["t_comp"] == o.tc
    # the compensation terms are rounding-sized
    assert np.abs(g["cx"]).max() <= 4 * np.spacing(np.abs(g["x"]).max())
    assert np.abs(g["cv"]).max() <= 4 * np.spacing(np.abs(g["v"]).max())


def test_compensated_symmetric_step_parity():
    _say("compensated symmetric step disc100")
    w = disc100()
    o = ho.State(w["mass"], w["x"], w["v"], 3)
    ho.init_derivs(o, eps2=w["eps2"])
    h = Hermite(8, len(w["mass"]), eps2=w["eps2"], compensated=True, device=DEV)
    st = h.state(w["mass"], w["x"], w["v"])
    h.init(st)
    for _ in range(20):
        do = ho.step_symmetric(o, 0.08, 4, eps2=w["eps2"], compensated=True)
        dg = h.step_symmetric(st, 0.08, 4)
        assert abs(dg / do - 1.0) <= 1e-12
    g = st.host()
    h.close()
    assert rel_max(g["x"], o.x) <= 1e-11 and rel_max(g["v"], o.v) <= 1e-11
    assert g["t"] == pytest.approx(o.t, rel=1e-13)


def _free_particle(compensated, steps=10000, dt=0.1):
    h = Hermite(4, 1, compensated=compensated, device=DEV)
    st = h.state([1.0], [[0.7], [0.0], [0.0]], [[1.0 / 3.0], [0.0], [0.0]])
    h.init(st)
    for _ in range(steps):
        h.step(st, dt, 1)
    d = st.host()
    h.close()
    inc = Fraction(float(np.float64(1.0 / 3.0) * dt))
    return d, abs(Fraction(float(d["x"][0, 0])) - (Fraction(0.7) + steps * inc))


def test_free_particle_on_gpu():
    # a = 0: each step adds fl(v dt) once; the exact sum is rational
    _say("compensated free particle")
    dc, err_c = _free_particle(True)
    dp, err_p = _free_particle(False)
    ulp = Fraction(float(np.spacing(dc["x"][0, 0])))
    assert err_c <= ulp
    assert err_p > 50 * ulp
    assert dc["t"] == 1000.0 and dp["t"] != 1000.0


def _kepler_worst_energy(compensated, orbits=4, dt=2.0 ** -5):
    w = kepler_two_body(e=0.1)
    h = Hermite(8, 2, eps2=1e-16, compensated=compensated, device=DEV)
    st = h.state(w["mass"], w["x"], w["v"])
    h.init(st)
    E0 = ho.energy(w["mass"], w["x"], w["v"], eps2=1e-16)
    worst = 0.0
    for _ in range(int(orbits * 2 * np.pi / dt)):
        h.step(st, dt, 3)
        d = st.host()
        worst = max(worst, abs(ho.energy(d["mass"], d["x"], d["v"], eps2=1e-16) / E0 - 1.0))
    h.close()
    return worst


def test_compensation_lowers_round_off_energy_error_on_gpu():
    # Sec. 3.2: 8th order at a step where truncation is below round-off
    _say("compensated kepler round-off")
    plain = _kepler_worst_energy(False)
    comp = _kepler_worst_energy(True)
    assert plain < 1e-14
    assert comp < 0.5 * plain


def test_compensated_checkpoint_resume_bitwise():
    _say("compensated checkpoint resume")
    w, _ = disc_path(300, 1)
    dt = 2 * np.pi / 2000
    h = Hermite(8, 300, compensated=True, device=DEV)
    a = h.state(w["mass"], w["x"], w["v"])
    h.init(a)
    for _ in range(6):
        h.step(a, dt, 3)
    b = h.state(w["mass"], w["x"], w["v"])
    h.init(b)
    for _ in range(3):
        h.step(b, dt, 3)
    c = h.restore(b.host())
    for _ in range(3):
        h.step(c, dt, 3)
    da, dc = a.host(), c.host()
    for k in ("x", "v", "cx", "cv"):
        assert np.array_equal(da[k], dc[k]), k
    assert da["t"] == dc["t"] and da["t_comp"] == dc["t_comp"]
    assert all(np.array_equal(p, q) for p, q in zip(da["derivs"], dc["derivs"]))
    h.close()


def test_compensated_needs_comp_array():
    _say("compensated without comp")
    w = kepler_two_body(e=0.5)
    h = Hermite(8, 2, compensated=True, device=DEV)
    st = h.state(w["mass"], w["x"], w["v"])
    st.c.comp = None
    with pytest.raises(HermiteError) as ei:
        h.init(st)
    assert ei.value.status == -1
    h.close()


# --- batched form -------------------------------------------------------------

def test_batched_compensated_matches_oracle():
    # three systems (Kepler 4-, 8th-order copies and a 5-body cluster) in one
    # compensated persistent launch against the oracle's compensated steps
    _say("batched compensated vs oracle")
    from paper_2006_02501_amd import BatchHermite

    kep = kepler_two_body(e=0.5)
    rng = np.random.default_rng(5)
    cl = dict(mass=np.concatenate([[1.0], rng.uniform(1e-6, 1e-4, 4)]),
              x=np.concatenate([np.zeros((3, 1)), rng.normal(size=(3, 4))], axis=1), v=np.zeros((3, 5)))
    r = np.sqrt((cl["x"][:, 1:] ** 2).sum(axis=0))
    cl["v"][:, 1:] = np.cross(np.array([0.0, 0.0, 1.0]), cl["x"][:, 1:].T).T / r ** 1.5
    systems = [kep, kep, cl]
    mass = np.concatenate([w["mass"] for w in systems])
    x = np.ascontiguousarray(np.concatenate([w["x"] for w in systems], axis=1))
    v = np.ascontiguousarray(np.concatenate([w["v"] for w in systems], axis=1))
    off = np.array([0, 2, 4, 9], dtype=np.int64)
    dts = np.array([kep["period"] / 200, kep["period"] / 150, 0.002])
    steps = 50
    bh = BatchHermite(8, off, compensated=True, device=DEV)
    st = bh.state(mass, x, v)
    bh.init(st)
    bh.run(st, dts, steps, 3)
    g = st.host()
    bh.close()
    for k, w in enumerate(systems):
        o = ho.State(w["mass"], w["x"], w["v"], 3)
        ho.init_derivs(o)
        for _ in range(steps):
            ho.step(o, dts[k], 3, compensated=True)
        sl = slice(off[k], off[k + 1])
        assert rel_max(g["x"][:, sl], o.x) <= 1e-11 and rel_max(g["v"][:, sl], o.v) <= 1e-11, k
    assert np.abs(g["cx"]).max() <= 4 * np.spacing(np.abs(g["x"]).max())


def test_batched_free_particles_exact():
    # 64 one-body systems (no force): each x is the rational sum of its
    # rounded increments; compensated within one ulp, plain far off
    _say("batched free particles")
    from paper_2006_02501_amd import BatchHermite

    k = 64
    rng = np.random.default_rng(9)
    x0 = rng.uniform(0.5, 2.0, k)
    v0 = rng.uniform(0.1, 1.0, k) / 3.0
    dt = 0.1
    steps = 10000
    res = {}
    for comp in (True, False):
        bh = BatchHermite(4, np.arange(k + 1, dtype=np.int64), compensated=comp, device=DEV)
        st = bh.state(np.ones(k), np.stack([x0, np.zeros(k), np.zeros(k)]), np.stack([v0, np.zeros(k), np.zeros(k)]))
        bh.init(st)
        bh.run(st, np.full(k, dt), steps, 1)
        res[comp] = st.host()["x"][0]
        bh.close()
    errs = {}
    for comp in (True, False):
        e = []
        for i in range(k):
            exact = Fraction(float(x0[i])) + steps * Fraction(float(np.float64(v0[i]) * dt))
            e.append(float(abs(Fraction(float(res[comp][i])) - exact) / Fraction(float(np.spacing(res[comp][i])))))
        errs[comp] = np.array(e)
    assert errs[True].max() <= 1.0, errs[True].max()
    assert errs[False].max() > 50.0, errs[False].max()


def test_batched_compensation_lowers_round_off():
    # Sec. 3.2 on the batched form: 16 copies of the e = 0.1 Kepler orbit,
    # 8th order, dt = 2^-5, 4 orbits, energy after every step
    _say("batched compensated kepler round-off")
    from paper_2006_02501_amd import BatchHermite

    w = kepler_two_body(e=0.1)
    k = 16
    mass = np.tile(w["mass"], k)
    x = np.ascontiguousarray(np.tile(w["x"], (1, k)))
    v = np.ascontiguousarray(np.tile(w["v"], (1, k)))
    off = np.arange(0, 2 * k + 1, 2, dtype=np.int64)
    dt = 2.0 ** -5
    worst = {}
    for comp in (False, True):
        bh = BatchHermite(8, off, eps2=1e-16, compensated=comp, device=DEV)
        st = bh.state(mass, x, v)
        bh.init(st)
        E0 = ho.energy(w["mass"], w["x"], w["v"], eps2=1e-16)
        wst = 0.0
        for _ in range(int(4 * 2 * np.pi / dt)):
            bh.run(st, np.full(k, dt), 1, 3)
            d = st.host()
            wst = max(wst, abs(ho.energy(d["mass"][:2], d["x"][:, :2], d["v"][:, :2], eps2=1e-16) / E0 - 1.0))
        bh.close()
        worst[comp] = wst
    assert worst[False] < 1e-14
    assert worst[True] < 0.5 * worst[False], worst


def test_batched_compensated_ring_bin_matches_oracle():
    # compensated 8th-order batched kernel (one sweep step in flight, the
    # iterate's x, v and compensation terms held in LDS between iterations)
    # on a bin that sweeps the whole wave as one ring (60 + 4 bodies)
    _say("batched compensated ring bin vs oracle")
    from paper_2006_02501_amd import BatchHermite
    from workloads import batch_systems

    wb = batch_systems()
    sizes = np.diff(wb["offsets"])
    want = [60, 4]
    mass, xs, vs, dts = [], [], [], []
    for n in want:
        s = int(np.nonzero(sizes == n)[0][0])
        lo = wb["offsets"][s]
        mass.append(wb["mass"][lo:lo + n])
        xs.append(wb["x"][:, lo:lo + n])
        vs.append(wb["v"][:, lo:lo + n])
        dts.append(wb["dt"][s])
    off = np.concatenate([[0], np.cumsum(want)]).astype(np.int64)
    mass = np.concatenate(mass)
    x = np.ascontiguousarray(np.concatenate(xs, axis=1))
    v = np.ascontiguousarray(np.concatenate(vs, axis=1))
    steps = 12
    bh = BatchHermite(8, off, compensated=True, device=DEV)
    st = bh.state(mass, x, v)
    bh.init(st)
    bh.run(st, np.array(dts), steps, 3)
    g = st.host()
    bh.close()
    for k in range(len(want)):
        sl = slice(off[k], off[k + 1])
        o = ho.State(mass[sl], x[:, sl], v[:, sl], 3)
        ho.init_derivs(o)
        for _ in range(steps):
            ho.step(o, dts[k], 3, compensated=True)
        assert rel_max(g["x"][:, sl], o.x) <= 1e-11 and rel_max(g["v"][:, sl], o.v) <= 1e-10, want[k]
