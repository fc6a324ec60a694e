"""GPU parity of the ensemble form (systems of 2..128 bodies, one workgroup
each, variable time-symmetric steps of Sec. 3.3 taken on the device) against
the oracle's step_symmetric loop: states, times, step counts and recorded
energies; chunked runs against one run; error paths."""
import sys

import numpy as np
import pytest

from oracle import hermite_oracle as ho
from paper_2006_02501_amd import EnsembleHermite, HermiteError
from parity_util import rel_max
from workloads import disc100, kepler_two_body

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _concat(systems):
    mass = np.concatenate([w["mass"] for w in systems])
    x = np.ascontiguousarray(np.concatenate([w["x"] for w in systems], axis=1))
    v = np.ascontiguousarray(np.concatenate([w["v"] for w in systems], axis=1))
    off = np.concatenate([[0], np.cumsum([len(w["mass"]) for w in systems])]).astype(np.int64)
    return mass, x, v, off


def _cluster(n, seed):
    rng = np.random.default_rng(seed)
    return dict(mass=rng.uniform(0.5, 1.5, n) / n, x=rng.normal(size=(3, n)), v=0.3 * rng.normal(size=(3, n)))


def _oracle_run(w, order, eta, n_iter, t_end, eps2, rec_from):
    st = ho.State(w["mass"], w["x"], w["v"], order // 2 - 1)
    ho.init_derivs(st, eps2=eps2)
    E0 = ho.energy(st.mass, st.x, st.v, eps2=eps2)
    rec, steps = [], 0
    while st.t < t_end:
        ho.step_symmetric(st, eta, n_iter, eps2=eps2)
        steps += 1
        if st.t > rec_from:
            rec.append((st.t, ho.energy(st.mass, st.x, st.v, eps2=eps2)))
    return st, E0, np.array(rec).reshape(-1, 2), steps


@pytest.mark.parametrize("order", [4, 6, 8])
def test_ensemble_matches_oracle(order):
    # one launch: a Kepler orbit (e = 0.7), the 100-body disc, a 7-body and a
    # 128-body softened cluster, and a Kepler orbit (e = 0.3) with a single
    # correction per step, each with its own eta and n
    _say("ensemble vs oracle order=%d" % order)
    kep = kepler_two_body(e=0.7, mean_anomaly=0.4)
    systems = [kep, disc100(), _cluster(7, 1), _cluster(128, 2), kepler_two_body(e=0.3, mean_anomaly=1.1)]
    etas = [0.05, 0.08, 0.1, 0.1, 0.05]
    iters = [4, 3, 2, 4, 1]
    t_ends = [0.3, 0.02, 0.5, 0.5, 0.3]
    eps2 = 1e-12
    mass, x, v, off = _concat(systems)
    eh = EnsembleHermite(order, off, eps2=eps2, device=DEV)
    st = eh.state(mass, x, v)
    eh.init(st, rec_cap=64)
    rec_from = [t / 2 for t in t_ends]
    res = eh.run(st, etas, t_ends, iters, rec_from=rec_from)
    g = st.host()
    for k, w in enumerate(systems):
        lo, hi = off[k], off[k + 1]
        o, E0, orec, steps = _oracle_run(w, order, etas[k], iters[k], t_ends[k], eps2, rec_from[k])
        r = res[k]
        assert r["steps"] == steps and r["failed"] == 0, (k, r, steps)
        assert r["t"] == pytest.approx(o.t, rel=1e-13)
        assert rel_max(g["x"][:, lo:hi], o.x) <= 1e-11 and rel_max(g["v"][:, lo:hi], o.v) <= 1e-11, k
        assert r["E0"] == pytest.approx(E0, rel=1e-13)
        assert r["records"] == len(orec)
        grec = eh.records(k, r["records"])
        assert np.allclose(grec[:, 0], orec[:, 0], rtol=1e-13, atol=0)
        assert np.allclose(grec[:, 1], orec[:, 1], rtol=1e-12, atol=0)
    eh.close()


def test_ensemble_init_matches_oracle():
    _say("ensemble init")
    systems = [kepler_two_body(e=0.5), disc100(), _cluster(65, 3)]
    mass, x, v, off = _concat(systems)
    eh = EnsembleHermite(8, off, eps2=1e-10, device=DEV)
    st = eh.state(mass, x, v)
    eh.init(st)
    g = st.host()
    for k, w in enumerate(systems):
        o = ho.State(w["mass"], w["x"], w["v"], 3)
        ho.init_derivs(o, eps2=1e-10)
        for q in range(6):
            assert rel_max(g["derivs"][q][:, off[k]:off[k + 1]], o.derivs[q]) <= 1e-11, (k, q)
    eh.close()


def test_ensemble_chunked_equals_single_run():
    _say("ensemble chunked")
    systems = [disc100(), kepler_two_body(e=0.3)]
    mass, x, v, off = _concat(systems)
    out = []
    for chunk in (None, 7):
        eh = EnsembleHermite(8, off, eps2=1e-12, device=DEV)
        st = eh.state(mass, x, v)
        eh.init(st, rec_cap=128)
        while True:
            res = eh.run(st, [0.08, 0.05], [0.05, 1.0], [3, 3], rec_from=[0.0, 0.5],
                         max_steps=chunk if chunk else 1 << 40)
            if all(r["t"] >= te for r, te in zip(res, [0.05, 1.0])):
                break
        out.append((st.host(), res, [eh.records(k, res[k]["records"]).copy() for k in range(2)]))
        eh.close()
    (a, ra, reca), (b, rb, recb) = out
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["v"], b["v"])
    assert all(np.array_equal(p, q) for p, q in zip(a["derivs"], b["derivs"]))
    assert [r["steps"] for r in ra] == [r["steps"] for r in rb] and [r["t"] for r in ra] == [r["t"] for r in rb]
    assert all(np.array_equal(p, q) for p, q in zip(reca, recb))


def test_ensemble_record_overflow_and_errors():
    _say("ensemble errors")
    w = disc100()
    mass, x, v, off = _concat([w])
    eh = EnsembleHermite(8, off, eps2=1e-12, device=DEV)
    st = eh.state(mass, x, v)
    eh.init(st, rec_cap=3)
    res = eh.run(st, 0.08, 0.03, 3, rec_from=0.0)
    assert res[0]["records"] == 3 and res[0]["rec_overflow"] == 1 and res[0]["steps"] > 3
    for bad in (dict(eta=0.0), dict(eta=float("nan")), dict(n_iter=0), dict(n_iter=65), dict(t_end=float("inf"))):
        kw = dict(eta=0.08, t_end=0.05, n_iter=3)
        kw.update(bad)
        with pytest.raises(HermiteError) as ei:
            eh.run(st, kw["eta"], kw["t_end"], kw["n_iter"])
        assert ei.value.status == -1, bad
    eh.close()
    # system sizes, precision
    for offs in ([0, 1], [0, 129], [0, 5, 5]):
        with pytest.raises(HermiteError):
            EnsembleHermite(8, np.array(offs), device=DEV)
    # no massive pair: the criterion is undefined, the system stops
    z = dict(mass=np.zeros(3), x=np.eye(3), v=np.zeros((3, 3)))
    mass, x, v, off = _concat([z, kepler_two_body(e=0.1)])
    eh = EnsembleHermite(4, off, device=DEV)
    st = eh.state(mass, x, v)
    eh.init(st)
    with pytest.raises(HermiteError) as ei:
        eh.run(st, 0.05, 1.0, 2)
    assert ei.value.status == -5
    g = st.host()
    assert np.array_equal(g["x"][:, :3], np.eye(3))
    eh.close()
