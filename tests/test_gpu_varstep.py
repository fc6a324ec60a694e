"""GPU parity of the variable, time-symmetric step (Sec. 3.3, Eq. 25) against
the oracle: the criterion H on ragged and multi-tile sizes (and at 2^20
bodies against Kepler's third law for a planted binary), whole steps with
their lengths, reversibility, the mixed-precision path within a bound derived
from its force error, and the error paths."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import hermite_oracle as ho
from paper_2006_02501_amd import Hermite, HermiteError
from parity_util import TOL_MIXED, disc_path, rel_max
from workloads import disc100, kepler_two_body

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# H = eta q^(-1/2): the GPU's q carries the refined reciprocal square root
# (<= 1.5 ulp), its cube (2 roundings), the mass sum and the product, and a
# differently ordered r^2 (3 roundings); |dH/H| = |dq/q|/2 + 2 roundings
# (sqrt, division) < 6 ulp.  The bar leaves a factor ~8.
TOL_H = 1e-14


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _criterion_pair(mass, x, eta, eps2, G=1.0):
    n = len(mass)
    h = Hermite(4, n, eps2=eps2, G=G, device=DEV)
    st = h.state(mass, x, np.zeros((3, n)))
    g = h.step_criterion(st, eta)
    h.close()
    return g, ho.step_criterion(mass, x, eta, G=G, eps2=eps2)


@pytest.mark.parametrize("n", [2, 3, 63, 257, 1000, 2050, 16384])
@pytest.mark.parametrize("eps2", [0.0, 1e-4])
def test_criterion_parity(n, eps2):
    _say("criterion n=%d eps2=%g" % (n, eps2))
    rng = np.random.default_rng(n)
    mass = rng.uniform(0.1, 1.0, n) * np.exp(rng.normal(size=n))
    x = rng.normal(size=(3, n))
    g, o = _criterion_pair(mass, x, 0.07, eps2, G=1.3)
    assert abs(g / o - 1.0) <= TOL_H, (g, o)


def test_criterion_parity_disc100():
    _say("criterion disc100")
    w = disc100()
    g, o = _criterion_pair(w["mass"], w["x"], 0.08, w["eps2"])
    assert abs(g / o - 1.0) <= TOL_H, (g, o)


@pytest.mark.parametrize("where", ["first", "last"])
def test_criterion_full_size_planted_binary(where):
    # 2^20 bodies of 1e-6 on a lattice of spacing 0.01 (every lattice pair:
    # q <= 2e-6 / 1e-6 = 2); one of them moved to ~1e-3 from another (q ~
    # 2e-6 / 1e-9 = 2000).  Kepler's third law then gives H for that binary:
    # eta (d^3 / (G 2m))^(1/2), d the stored separation (an exact difference).
    _say("criterion 2^20 planted binary (%s)" % where)
    side = (64, 128, 128)
    idx = np.indices(side).reshape(3, -1).astype(np.float64) * 0.01
    n = idx.shape[1]
    mass = np.full(n, 1e-6)
    x = np.ascontiguousarray(idx)
    a, b = (0, 1) if where == "first" else (n - 2, n - 1)
    x[:, b] = x[:, a] + np.array([1e-3, 0.0, 0.0])
    h = Hermite(4, n, device=DEV)
    st = h.state(mass, x, np.zeros((3, n)))
    g = h.step_criterion(st, 0.05)
    h.close()
    d = x[0, b] - x[0, a]
    expect = 0.05 * math.sqrt(d ** 3 / 2e-6)
    assert abs(g / expect - 1.0) <= TOL_H, (g, expect)


def _run_pair(order, w, eta, n_iter, steps, eps2=0.0, precision="fp64", direction=1.0, launch=None):
    p = order // 2 - 1
    o = ho.State(w["mass"], w["x"], w["v"], p)
    ho.init_derivs(o, eps2=eps2)
    n = len(w["mass"])
    h = Hermite(order, n, precision=precision, eps2=eps2, device=DEV)
    if launch is not None:
        h.set_launch(*launch)
    st = h.state(w["mass"], w["x"], w["v"])
    h.init(st)
    dts = []
    for _ in range(steps):
        do = ho.step_symmetric(o, eta, n_iter, eps2=eps2, direction=direction)
        dg = h.step_symmetric(st, eta, n_iter, direction=direction)
        dts.append((dg, do))
    d = st.host()
    h.close()
    return o, d, np.array(dts)


@pytest.mark.parametrize("order", [4, 6, 8])
def test_symmetric_step_parity_kepler(order):
    _say("symmetric step kepler order=%d" % order)
    w = kepler_two_body(e=0.7, mean_anomaly=0.4)
    o, g, dts = _run_pair(order, w, 0.05, 4, 1)
    assert abs(dts[0, 0] / dts[0, 1] - 1.0) <= TOL_H
    assert rel_max(g["x"], o.x) <= 1e-13 and rel_max(g["v"], o.v) <= 1e-13
    o, g, dts = _run_pair(order, w, 0.05, 4, 40)
    assert np.max(np.abs(dts[:, 0] / dts[:, 1] - 1.0)) <= 1e-12
    assert rel_max(g["x"], o.x) <= 1e-11 and rel_max(g["v"], o.v) <= 1e-11
    assert g["t"] == pytest.approx(o.t, rel=1e-12)
    # backwards
    o, g, dts = _run_pair(order, w, 0.05, 4, 5, direction=-1.0)
    assert np.all(dts[:, 0] < 0.0)
    assert rel_max(g["x"], o.x) <= 1e-12 and rel_max(g["v"], o.v) <= 1e-12


@pytest.mark.parametrize("order,n_iter", [(8, 1), (8, 2), (8, 3), (8, 4), (6, 2), (4, 4)])
def test_symmetric_step_parity_disc100(order, n_iter):
    # the paper's disc test set-up (eta = 0.08, eps = 1e-6), 30 steps
    _say("symmetric step disc100 order=%d n=%d" % (order, n_iter))
    w = disc100()
    o, g, dts = _run_pair(order, w, 0.08, n_iter, 30, eps2=w["eps2"])
    assert np.max(np.abs(dts[:, 0] / dts[:, 1] - 1.0)) <= 1e-12
    assert rel_max(g["x"], o.x) <= 1e-11 and rel_max(g["v"], o.v) <= 1e-11
    for k in range(order // 2):
        assert rel_max(g["derivs"][k], o.derivs[k]) <= 1e-9, k


def test_symmetric_step_reversible_on_gpu():
    # converged iterations: a step backwards from the end returns to the start
    _say("symmetric step reversibility")
    w = kepler_two_body(e=0.7, mean_anomaly=0.4)
    h = Hermite(8, 2, device=DEV)
    st = h.state(w["mass"], w["x"], w["v"])
    h.init(st)
    d0 = st.host()
    f = h.step_symmetric(st, 0.1, 12)
    b = h.step_symmetric(st, 0.1, 12, direction=-1.0)
    d1 = st.host()
    h.close()
    assert b == pytest.approx(-f, rel=1e-13)
    assert np.max(np.abs(d1["x"] - d0["x"])) < 1e-13 and np.max(np.abs(d1["v"] - d0["v"])) < 1e-13
    assert abs(d1["t"]) < 1e-15


@pytest.mark.parametrize("launch", [(1, 1, 0, 4), (2, 3, 0, 4), (1, 64, 1, 4), (2, 0, 1, 4), (1, 5, 1, 16),
                                    (1, 0, 2, 4)])
@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_fused_rate_in_every_launch_shape(launch, precision):
    # FP64 and split evaluations take the pair rate along (one maximum per
    # workgroup); the step length must not depend on the launch shape
    _say("fused rate launch=%s %s" % (launch, precision))
    w = disc100()
    eps2 = w["eps2"]
    o = ho.State(w["mass"], w["x"], w["v"], 3)
    ho.init_derivs(o, eps2=eps2)
    h = Hermite(8, len(w["mass"]), precision=precision, eps2=eps2, device=DEV)
    h.set_launch(*launch)
    st = h.state(w["mass"], w["x"], w["v"])
    h.init(st)
    for _ in range(3):
        do = ho.step_symmetric(o, 0.08, 3, eps2=eps2)
        dg = h.step_symmetric(st, 0.08, 3)
        assert abs(dg / do - 1.0) <= (1e-13 if precision == "fp64" else 1e-9), (dg, do)
    g = st.host()
    h.close()
    if precision == "fp64":
        assert rel_max(g["x"], o.x) <= 1e-13 and rel_max(g["v"], o.v) <= 1e-13


@pytest.mark.parametrize("nb", [101, 700])
def test_fused_rate_pairs_once(nb):
    # the every-pair-once evaluation takes the pair rate along too (one
    # maximum per super-block pair): the same steps as the oracle's
    _say("fused rate pairs-once n=%d" % nb)
    w = disc100() if nb == 101 else dict(disc_path(nb, 1)[0], eps2=1e-8)
    eps2 = w["eps2"]
    o = ho.State(w["mass"], w["x"], w["v"], 3)
    ho.init_derivs(o, eps2=eps2)
    h = Hermite(8, len(w["mass"]), eps2=eps2, device=DEV)
    h.set_launch(1, 0, 2, 4)
    st = h.state(w["mass"], w["x"], w["v"])
    h.init(st)
    for _ in range(3):
        do = ho.step_symmetric(o, 0.08, 3, eps2=eps2)
        dg = h.step_symmetric(st, 0.08, 3)
        assert abs(dg / do - 1.0) <= 1e-13, (dg, do)
    g = st.host()
    h.close()
    assert rel_max(g["x"], o.x) <= 1e-13 and rel_max(g["v"], o.v) <= 1e-13


@pytest.mark.parametrize("order,n", [(4, 9217), (8, 9217), (4, 33000)])
def test_pairs_symmetric_step_matches_lds(order, n):
    # n = 9217: one every-pair-once launch of whole items (one workgroup per
    # item at both orders) that carries the rate; n = 33000: beyond 32768
    # bodies the evaluation runs in chunks and keeps no rate, so the variable
    # step takes the separate criterion pass.  Either way the steps must
    # match those of the LDS kernel (which fuses the rate).
    _say("symmetric step, pairs vs LDS, order=%d n=%d" % (order, n))
    w, _ = disc_path(n, 1)
    out = {}
    for name, launch in (("lds", (2, 4, 0, 4)), ("pairs", (1, 0, 2, 4))):
        h = Hermite(order, n, eps2=1e-10, device=DEV)
        h.set_launch(*launch)
        st = h.state(w["mass"], w["x"], w["v"])
        h.init(st)
        dts = [h.step_symmetric(st, 0.05, 3) for _ in range(3)]
        out[name] = (np.array(dts), st.host())
        h.close()
    (da, ga), (db, gb) = out["lds"], out["pairs"]
    assert np.max(np.abs(db / da - 1.0)) <= 1e-13, (da, db)
    assert rel_max(gb["x"], ga["x"]) <= 1e-13 and rel_max(gb["v"], ga["v"]) <= 1e-13


@pytest.mark.parametrize("launch", [None, (1, 0, 2, 4)])
def test_mixed_symmetric_step_within_force_bound(launch):
    # The mixed evaluation's relative force error delta (<= 1e-6, the bar of
    # the mixed evaluation on a) moves each iterate's x by <= delta a dt^2 / 2
    # and v by <= delta a dt; the step's length follows H ~ r^(3/2) of the
    # tightest pair, so |d dt / dt| <= 1.5 (2 delta a dt^2 / 2) / r_pair per
    # step.  Over the run the two states also sit at times that differ by
    # |t_gpu - t_oracle|, which moves x by v_max |dt| and v by a_max |dt|.
    # (a_max = G M / r_min^2 with r_min the smallest distance to the central
    # mass; v_max = (2 G M / r_min)^(1/2).)  All bounds carry a factor 2.
    # The default launch takes the criterion from a separate FP64 pass, every
    # pair once from the evaluation's FP64 differences.
    _say("mixed symmetric step disc100 launch=%s" % (launch,))
    w = disc100()
    steps = 5
    o, g, dts = _run_pair(8, w, 0.08, 3, steps, eps2=w["eps2"], precision="mixed", launch=launch)
    delta = TOL_MIXED[0]
    rc = np.sqrt(np.sum((w["x"][:, 1:] - w["x"][:, :1]) ** 2, axis=0))
    r_min = 0.9 * rc.min()
    a_max, v_max = 1.0 / r_min ** 2, math.sqrt(2.0 / r_min)
    dt = np.abs(dts[:, 1]).max()
    rel_dt = np.max(np.abs(dts[:, 0] / dts[:, 1] - 1.0))
    assert rel_dt <= 2.0 * steps * 1.5 * delta * a_max * dt ** 2 / r_min, rel_dt
    tdiff = abs(g["t"] - o.t)
    dx = np.abs(g["x"] - o.x).max()
    dv = np.abs(g["v"] - o.v).max()
    assert dx <= 2.0 * (steps * delta * a_max * dt ** 2 / 2 + v_max * tdiff), dx
    assert dv <= 2.0 * (steps * delta * a_max * dt + a_max * tdiff), dv


def test_variable_step_errors():
    _say("variable step errors")
    w = kepler_two_body(e=0.5)
    h = Hermite(8, 4, device=DEV)
    st = h.state(w["mass"], w["x"], w["v"])
    with pytest.raises(HermiteError) as ei:
        h.step_symmetric(st, 0.1, 2)
    assert ei.value.status == -6                     # not initialised
    h.init(st)
    for eta, n_iter, direction in ((0.0, 2, 1.0), (-0.1, 2, 1.0), (float("nan"), 2, 1.0), (0.1, 0, 1.0),
                                   (0.1, 2, 0.5), (0.1, 2, 0.0)):
        with pytest.raises(HermiteError) as ei:
            h.step_symmetric(st, eta, n_iter, direction)
        assert ei.value.status == -1, (eta, n_iter, direction)
    one = h.state(w["mass"][:1], w["x"][:, :1], w["v"][:, :1])
    h.init(one)
    with pytest.raises(HermiteError) as ei:
        h.step_criterion(one, 0.1)
    assert ei.value.status == -1
    with pytest.raises(HermiteError) as ei:
        h.step_symmetric(one, 0.1, 2)
    assert ei.value.status == -1
    # no massive pair: H is not finite; the state is left as it was
    zero = h.state(np.zeros(3), np.eye(3), np.zeros((3, 3)))
    h.init(zero)
    with pytest.raises(HermiteError) as ei:
        h.step_criterion(zero, 0.1)
    assert ei.value.status == -5
    with pytest.raises(HermiteError) as ei:
        h.step_symmetric(zero, 0.1, 2)
    assert ei.value.status == -5
    d = zero.host()
    assert np.array_equal(d["x"], np.eye(3)) and np.array_equal(d["v"], np.zeros((3, 3))) and d["t"] == 0.0
    # coincident bodies without softening: H = 0, same
    co = h.state(np.ones(2), np.zeros((3, 2)), np.ones((3, 2)))
    h.init(co)
    with pytest.raises(HermiteError) as ei:
        h.step_symmetric(co, 0.1, 2)
    assert ei.value.status == -5
    d = co.host()
    assert np.array_equal(d["x"], np.zeros((3, 2))) and np.array_equal(d["v"], np.ones((3, 2))) and d["t"] == 0.0
    # a criterion that fails only at the predicted end point (H_- is finite;
    # the prediction for dt = H_- overflows the squared separation, so the
    # rate there is 0 and H_+ is not finite): the step fails with the state
    # left as it was, for one correction and for several
    for n_iter in (1, 2, 3):
        fast = h.state(np.ones(2), np.array([[-0.5, 0.5], [0.0, 0.0], [0.0, 0.0]]),
                       np.array([[-1e300, 1e300], [0.0, 0.0], [0.0, 0.0]]))
        h.init(fast)
        d0 = fast.host()
        with pytest.raises(HermiteError) as ei:
            h.step_symmetric(fast, 0.1, n_iter)
        assert ei.value.status == -5, n_iter
        d = fast.host()
        assert np.array_equal(d["x"], d0["x"]) and np.array_equal(d["v"], d0["v"]) and d["t"] == 0.0, n_iter
    # the context still works afterwards
    dt = h.step_symmetric(st, 0.1, 2)
    assert dt > 0.0
    h.close()
