"""GPU parity of the split-precision evaluation (the paper's suggestion of
lower precision for the higher-order terms, Sec. 4): a and adot bitwise equal
to the FP64 path's in every launch shape, a^(2) and a^(3) within the mixed
bars against the oracle, and whole steps within a bound derived from those
bars."""
import sys

import numpy as np
import pytest
import torch

from oracle import hermite_oracle as ho
from paper_2006_02501_amd import Hermite
from parity_util import TOL_FP64, TOL_MIXED, deriv_error, disc_path, random_path

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

SHAPES = [(1, 1, 0, 4), (2, 3, 0, 4), (1, 64, 1, 4), (2, 0, 1, 4), (1, 3, 1, 16), (1, 0, 1, 16), (1, 0, 2, 4)]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _ok(err, tol):
    """err [m][n] against a tolerance per row."""
    return bool(np.all(np.asarray(err).max(axis=1) <= np.asarray(tol)))


def _eval_gpu(order, mass, path, precision, eps2=0.0, G=1.0, launch=None):
    p = order // 2 - 1
    n = len(mass)
    h = Hermite(order, n, precision=precision, eps2=eps2, G=G, device=DEV)
    st = h.state(mass, path[0], path[1])
    for k in range(p + 1):
        st.pred[k].copy_(torch.as_tensor(np.asarray(path[k], dtype=np.float64).reshape(3, n)))
    if launch is not None:
        h.set_launch(*launch)
    h.force_derivs(st)
    out = st.eval.cpu().numpy()
    h.close()
    return out


@pytest.mark.parametrize("order", [6, 8])
@pytest.mark.parametrize("launch", SHAPES)
def test_split_low_orders_bitwise_fp64(order, launch):
    _say("split vs fp64 bitwise order=%d launch=%s" % (order, launch))
    p = order // 2 - 1
    w, path = disc_path(1500, p)
    s = _eval_gpu(order, w["mass"], path, "split", launch=launch)
    f = _eval_gpu(order, w["mass"], path, "fp64", launch=launch)
    assert np.array_equal(s[:2], f[:2])
    o, mag, nat = ho.pair_derivs(w["mass"], path, K=p, with_mag=True, with_scale=True)
    err = deriv_error(s, o, mag, nat)
    assert _ok(err, np.concatenate([[TOL_FP64, TOL_FP64], TOL_MIXED[2:p + 1]]))


@pytest.mark.parametrize("order", [6, 8])
@pytest.mark.parametrize("n", [2, 63, 257, 1000, 2050])
def test_split_disc(order, n):
    _say("split disc order=%d n=%d" % (order, n))
    p = order // 2 - 1
    w, path = disc_path(n, p)
    o, mag, nat = ho.pair_derivs(w["mass"], path, K=p, with_mag=True, with_scale=True)
    g = _eval_gpu(order, w["mass"], path, "split")
    assert deriv_error(g[:2], o[:2], mag[:2]).max() <= TOL_FP64
    assert _ok(deriv_error(g, o, mag, nat)[2:], TOL_MIXED[2:p + 1])


@pytest.mark.parametrize("order", [6, 8])
def test_split_random_softened(order):
    _say("split random softened order=%d" % order)
    rng = np.random.default_rng(order + 100)
    p = order // 2 - 1
    mass, path = random_path(rng, 777, p)
    o, mag, nat = ho.pair_derivs(mass, path, K=p, G=0.7, eps2=1e-3, with_mag=True, with_scale=True)
    g = _eval_gpu(order, mass, path, "split", eps2=1e-3, G=0.7)
    assert deriv_error(g[:2], o[:2], mag[:2]).max() <= TOL_FP64
    assert _ok(deriv_error(g, o, mag, nat)[2:], TOL_MIXED[2:p + 1])


@pytest.mark.parametrize("launch", [None, (1, 64, 1, 4), (1, 0, 2, 4)])
def test_split_full_size_sampled(launch):
    # the 16k disc at its full size, 192 sampled i, in the default launch shape
    # and in the one the benchmark times
    _say("split full size 16384", launch)
    w, path = disc_path(16384, 3)
    rng = np.random.default_rng(16)
    il = np.sort(rng.choice(16384, 192, replace=False))
    il[0], il[-1] = 0, 16383
    o, mag, nat = ho.pair_derivs(w["mass"], path, K=3, i_list=il, with_mag=True, with_scale=True)
    g = _eval_gpu(8, w["mass"], path, "split", launch=launch)[:, :, il]
    assert deriv_error(g[:2], o[:2], mag[:2]).max() <= TOL_FP64
    assert _ok(deriv_error(g, o, mag, nat)[2:], TOL_MIXED[2:])


def test_split_is_fp64_at_fourth_order():
    _say("split 4th order")
    w, path = disc_path(700, 1)
    assert np.array_equal(_eval_gpu(4, w["mass"], path, "split"), _eval_gpu(4, w["mass"], path, "fp64"))


def test_split_step_within_derived_bound():
    # Only a^(2), a^(3) differ from FP64, by <= delta_k D_k (the mixed bars on
    # their scale D_k = max(|a^(k)|, 0.1 S_k, N_k)).  In the 8th-order
    # corrector they enter v with the weights 1/84 dt^3 and 1/1680 dt^4 (times
    # the sum of both ends), so one correction moves v by <= B = 2 (delta_2
    # D_2 dt^3 / 84 + delta_3 D_3 dt^4 / 1680) per particle; over s steps v by
    # <= s B and x by <= s^2 B dt.  The bound carries a factor 2 for the
    # iterate-to-iterate feedback.
    _say("split step bound")
    w, path = disc_path(700, 3)
    dt = 2 * np.pi / 2000
    steps = 5
    o3, mag, nat = ho.pair_derivs(w["mass"], path, K=3, with_mag=True, with_scale=True)
    D = np.maximum(np.maximum(np.sqrt((o3 * o3).sum(axis=1)), 0.1 * mag), nat)
    d2, d3 = TOL_MIXED[2], TOL_MIXED[3]
    B = 2.0 * (d2 * D[2] * dt ** 3 / 84.0 + d3 * D[3] * dt ** 4 / 1680.0)   # per particle
    # the corrector weights used above are the 8th-order velocity ones
    cv = [float(c) for c in ho.endpoint_coefficients(3)]
    assert abs(cv[2]) == 1.0 / 84.0 and abs(cv[3]) == 1.0 / 1680.0
    o = ho.State(w["mass"], w["x"], w["v"], 3)
    ho.init_derivs(o)
    h = Hermite(8, 700, precision="split", device=DEV)
    st = h.state(w["mass"], w["x"], w["v"])
    h.init(st)
    for _ in range(steps):
        ho.step(o, dt, 3)
        h.step(st, dt, 3)
    g = st.host()
    h.close()
    dv = np.max(np.abs(g["v"] - o.v), axis=0)
    dx = np.max(np.abs(g["x"] - o.x), axis=0)
    floor = 1e-13 * np.abs(o.v).max()
    assert np.all(dv <= 2.0 * steps * B + floor), np.max(dv / (steps * B + floor))
    assert np.all(dx <= 2.0 * steps ** 2 * B * dt + 1e-13 * np.abs(o.x).max())
