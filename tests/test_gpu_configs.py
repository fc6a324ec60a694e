"""GPU parity at the full sizes of the cluster and large-disc workloads
(sampled i-particles, in the launch configuration the library picks by
default), plus the 64-body ring over its full 10-orbit run.

The evaluation path's a (and adot) are analytic fields of the right size --
the Plummer mean field for the cluster, the central body's Kepler field for
the disc -- so no input of the oracle comes from the HIP path."""
import sys

import numpy as np
import pytest
import torch

from oracle import hermite_oracle as ho
from paper_2006_02501_amd import Hermite
from parity_util import TOL_FP64, TOL_MIXED, deriv_error, rel_max, within
from workloads import large_disc, plummer_cluster, ring64

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _gpu_eval(order, w, path, precision, eps2, launch=None):
    p = order // 2 - 1
    n = len(w["mass"])
    h = Hermite(order, n, precision=precision, eps2=eps2, device=DEV)
    if launch is not None:
        h.set_launch(*launch)
    st = h.state(w["mass"], w["x"], w["v"])
    for k in range(p + 1):
        st.pred[k].copy_(torch.as_tensor(np.ascontiguousarray(path[k])))
    h.force_derivs(st)
    out = st.eval.cpu().numpy()
    h.close()
    return out


@pytest.fixture(scope="module")
def cluster():
    return plummer_cluster()


@pytest.mark.parametrize("launch", [None, (1, 0, 2, 4)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_plummer_cluster_full_size(cluster, precision, launch):
    # 131072 stars + a central mass 0.01, 6th order (a, adot, a^(2)), eps = 1e-4;
    # the default launch and every pair once (in chunks)
    _say("plummer cluster N=%d %s launch=%s" % (len(cluster["mass"]), precision, launch))
    w = cluster
    ap = 3.0 * np.pi / 16.0
    x = w["x"]
    a_mean = -x * (np.sum(x * x, axis=0) + ap * ap) ** -1.5
    path = [w["x"], w["v"], a_mean]
    rng = np.random.default_rng(2)
    il = np.sort(rng.choice(len(w["mass"]), 256, replace=False))
    il[-1] = len(w["mass"]) - 1               # the central mass
    o, mag, nat = ho.pair_derivs(w["mass"], path, K=2, eps2=w["eps2"], i_list=il, with_mag=True, with_scale=True)
    g = _gpu_eval(6, w, path, precision, w["eps2"], launch)[:, :, il]
    if precision == "fp64":
        err = deriv_error(g, o, mag)
        assert within(err, TOL_FP64), err.max(axis=1)
    else:
        err = deriv_error(g, o, mag, nat)
        assert within(err, TOL_MIXED), err.max(axis=1)
    _say("  max err per order", err.max(axis=1))


@pytest.fixture(scope="module")
def big_disc():
    return large_disc()


@pytest.mark.parametrize("launch", [None, (1, 0, 2, 4)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_large_disc_full_size(big_disc, precision, launch):
    # 1048576 bodies, 8th order (a .. a^(3)), one evaluation, 128 sampled i;
    # the default launch and every pair once (in chunks)
    _say("large disc N=%d %s launch=%s" % (len(big_disc["mass"]), precision, launch))
    w = big_disc
    x, v = w["x"], w["v"]
    r2 = np.sum(x * x, axis=0)
    rv = np.sum(x * v, axis=0)
    a_kep = -x * r2 ** -1.5
    j_kep = -v * r2 ** -1.5 + 3.0 * x * rv * r2 ** -2.5
    path = [x, v, a_kep, j_kep]
    rng = np.random.default_rng(4)
    il = np.sort(rng.choice(len(w["mass"]), 128, replace=False))
    il[0] = 0
    o, mag, nat = ho.pair_derivs(w["mass"], path, K=3, i_list=il, with_mag=True, with_scale=True)
    g = _gpu_eval(8, w, path, precision, 0.0, launch)[:, :, il]
    if precision == "fp64":
        err = deriv_error(g, o, mag)
        assert within(err, TOL_FP64), err.max(axis=1)
    else:
        err = deriv_error(g, o, mag, nat)
        assert within(err, TOL_MIXED), err.max(axis=1)
    _say("  max err per order", err.max(axis=1))


def test_ring64_ten_orbits():
    # 4th order, P(EC)^2, dt = 2 pi / 1000, 10 orbits (10^4 steps) on the GPU
    # against the oracle; energy stays bounded.
    _say("ring64 10 orbits")
    w = ring64()
    steps = w["steps"]
    h = Hermite(4, 64, device=DEV)
    st = h.state(w["mass"], w["x"], w["v"])
    h.init(st)
    E0 = ho.energy(w["mass"], w["x"], w["v"])
    for _ in range(steps):
        h.step(st, w["dt"], w["n_iter"])
    g = st.host()
    h.close()
    o = ho.State(w["mass"], w["x"], w["v"], 1)
    ho.init_derivs(o)
    for _ in range(steps):
        ho.step(o, w["dt"], w["n_iter"])
    E1 = ho.energy(g["mass"], g["x"], g["v"])
    assert rel_max(g["x"], o.x) <= 1e-9 and rel_max(g["v"], o.v) <= 1e-9
    assert abs(E1 / E0 - 1.0) < 1e-10
