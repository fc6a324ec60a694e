"""The paper's iteration-count sweep (Sec. 3.1, Fig. 4) on the batched GPU
path: the Kepler orbit (a = 1, e = 0.1, planet 1e-3, dt = 2^-4, eps = 1e-8)
integrated for 2000 orbital periods with n = 1, 2, 3, 4 side by side, one
persistent launch per order with a per-system iteration count.  Also the
parity of per-system counts with uniform ones (bitwise) and with the oracle."""
import sys

import numpy as np
import pytest

from oracle import hermite_oracle as ho
from paper_2006_02501_amd import BatchHermite
from parity_util import rel_max
from workloads import kepler_two_body

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
EPS2 = 1e-16
DT = 2.0 ** -4


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _copies(k, w):
    mass = np.tile(w["mass"], k)
    x = np.ascontiguousarray(np.tile(w["x"], (1, k)))
    v = np.ascontiguousarray(np.tile(w["v"], (1, k)))
    return mass, x, v, np.arange(0, 2 * k + 1, 2, dtype=np.int64)


def _pair_energy(m, x, v):
    # two bodies per system: kinetic - G m1 m2 / (r^2 + eps^2)^(1/2), per system
    m = m.reshape(-1, 2)
    x = x.reshape(3, -1, 2)
    v = v.reshape(3, -1, 2)
    kin = 0.5 * np.sum(m * np.sum(v * v, axis=0), axis=1)
    r2 = np.sum((x[:, :, 1] - x[:, :, 0]) ** 2, axis=0)
    return kin - m[:, 0] * m[:, 1] / np.sqrt(r2 + EPS2)


@pytest.mark.parametrize("order", [4, 6, 8])
def test_per_system_iterations_match_uniform_runs(order):
    # a bin with n = 1..4 gives, for each system, the bits of a run with that
    # n everywhere; and the oracle's steps
    _say("per-system n_iter order=%d" % order)
    w = kepler_two_body(e=0.1)
    mass, x, v, off = _copies(4, w)
    steps = 50
    bh = BatchHermite(order, off, eps2=EPS2, device=DEV)
    st = bh.state(mass, x, v)
    bh.init(st)
    bh.run(st, np.full(4, DT), steps, [1, 2, 3, 4])
    mixed = st.host()
    bh.close()
    p = order // 2 - 1
    for n in (1, 2, 3, 4):
        bu = BatchHermite(order, off, eps2=EPS2, device=DEV)
        su = bu.state(mass, x, v)
        bu.init(su)
        bu.run(su, np.full(4, DT), steps, n)
        uni = su.host()
        bu.close()
        sl = slice(2 * (n - 1), 2 * n)
        assert np.array_equal(mixed["x"][:, sl], uni["x"][:, sl]) and np.array_equal(mixed["v"][:, sl], uni["v"][:, sl])
        o = ho.State(w["mass"], w["x"], w["v"], p)
        ho.init_derivs(o, eps2=EPS2)
        for _ in range(steps):
            ho.step(o, DT, n, eps2=EPS2)
        assert rel_max(mixed["x"][:, sl], o.x) <= 1e-11 and rel_max(mixed["v"][:, sl], o.v) <= 1e-11


@pytest.fixture(scope="module")
def sweep():
    # 2000 periods, energy sampled every 997 steps (9.92 periods, so the
    # samples walk through the orbital phase)
    w = kepler_two_body(e=0.1)
    period = w["period"]
    total = int(round(2000 * period / DT))
    per = 997
    chunks = total // per
    out = {}
    for order in (4, 6, 8):
        mass, x, v, off = _copies(4, w)
        bh = BatchHermite(order, off, eps2=EPS2, device=DEV)
        st = bh.state(mass, x, v)
        bh.init(st)
        E0 = _pair_energy(mass, x, v)
        rec = []
        for _ in range(chunks):
            bh.run(st, np.full(4, DT), per, [1, 2, 3, 4])
            d = st.host()
            rec.append(np.abs(_pair_energy(d["mass"], d["x"], d["v"]) / E0 - 1.0))
        bh.close()
        out[order] = np.array(rec)          # [chunks][n = 1..4]
        _say("order %d: |dE/E| last sample n=1..4: %s; max: %s" % (order, rec[-1], np.max(rec, axis=0)))
    return out


@pytest.mark.parametrize("order", [4, 6, 8])
def test_fig4_claims(sweep, order):
    dE = sweep[order]
    worst = dE.max(axis=0)
    early = np.median(dE[:20], axis=0)
    late = np.median(dE[-20:], axis=0)
    # n = 2 is far better than n = 1 (orders of magnitude)
    assert worst[1] < 1e-2 * worst[0], worst
    # n = 3 and n = 4 nearly identical
    assert worst[3] < 3.0 * worst[2] and worst[2] < 3.0 * worst[3], worst
    # n = 1 drifts secularly over the 2000 orbits
    assert late[0] > 3.0 * early[0], (early, late)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_per_system_iterations_in_both_sweeps(precision):
    # Per-system counts in bins of both sweep kinds of the batched
    # evaluation: a whole-wave ring (60 + 4 bodies) and per-system rings
    # (40 + 24).  Pairs across systems count zero, so each system gets the
    # bits of a run with its own n everywhere.
    from workloads import batch_systems

    _say("per-system n_iter in ring and segment bins %s" % precision)
    wb = batch_systems()
    sizes = np.diff(wb["offsets"])
    want, counts = [60, 4, 40, 24], [3, 1, 4, 2]
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
    dts = np.array(dts)
    steps = 12

    def run(n_iter):
        bh = BatchHermite(8, off, precision=precision, device=DEV)
        st = bh.state(mass, x, v)
        bh.init(st)
        bh.run(st, dts, steps, n_iter)
        d = st.host()
        bh.close()
        return d

    mixed = run(counts)
    for k, n in enumerate(counts):
        uni = run(n)
        sl = slice(off[k], off[k + 1])
        assert np.array_equal(mixed["x"][:, sl], uni["x"][:, sl]), (want[k], n)
        assert np.array_equal(mixed["v"][:, sl], uni["v"][:, sl]), (want[k], n)
    if precision == "fp64":
        # the ring bin's 60-body system against the oracle
        o = ho.State(mass[:60], x[:, :60], v[:, :60], 3)
        ho.init_derivs(o)
        for _ in range(steps):
            ho.step(o, dts[0], 3)
        assert rel_max(mixed["x"][:, :60], o.x) <= 1e-11 and rel_max(mixed["v"][:, :60], o.v) <= 1e-10
