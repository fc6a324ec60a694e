"""The evaluation of an i-range (hermite_force_derivs_range): one GPU's share
of an evaluation divided among GPUs by i.  Against the full evaluation in the
same launch shape (bitwise with a fixed j-split), positions outside the range
untouched, and the per-GPU shape of an 8-way division of the 1M-body disc
against the oracle on sampled i.  The path's a and adot are analytic fields
(the central body's Kepler field), so no oracle input comes from the HIP
path."""
import sys

import numpy as np
import pytest
import torch

from oracle import hermite_oracle as ho
from paper_2006_02501_amd import Hermite, HermiteError
from parity_util import TOL_FP64, TOL_MIXED, deriv_error, within
from workloads import disc16k, large_disc

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _kepler_path(w):
    x, v = w["x"], w["v"]
    r2 = np.sum(x * x, axis=0)
    rv = np.sum(x * v, axis=0)
    return [x, v, -x * r2 ** -1.5, -v * r2 ** -1.5 + 3.0 * x * rv * r2 ** -2.5]


def _ctx(order, w, path, precision, launch):
    p = order // 2 - 1
    h = Hermite(order, len(w["mass"]), precision=precision, device=DEV)
    h.set_launch(*launch)
    st = h.state(w["mass"], w["x"], w["v"])
    for k in range(p + 1):
        st.pred[k].copy_(torch.as_tensor(np.ascontiguousarray(path[k])))
    return h, st


# one-sided shapes (i_per_thread, j_split, j_source, wg_waves), fixed splits
SHAPES = [(1, 4, 0, 4), (2, 3, 0, 4), (1, 8, 1, 4), (2, 2, 1, 4), (3, 4, 1, 4), (4, 1, 1, 4), (1, 5, 1, 16)]


@pytest.mark.parametrize("launch", SHAPES)
@pytest.mark.parametrize("precision", ["fp64", "mixed", "split"])
def test_range_bitwise_as_full_evaluation(precision, launch):
    n = 3001
    w = disc16k(n)
    path = _kepler_path(w)
    h, st = _ctx(8, w, path, precision, launch)
    h.force_derivs(st)
    full = st.eval.clone()
    for i0, ni in [(0, n), (0, 1), (37, 1000), (n - 5, 5), (1290, 1), (700, 1711)]:
        _say("range %s %s [%d, %d)" % (precision, launch, i0, i0 + ni))
        st.eval.fill_(float("nan"))
        h.force_derivs_range(st, i0, ni)
        g = st.eval
        assert torch.equal(g[:, :, i0:i0 + ni], full[:, :, i0:i0 + ni]), (i0, ni)
        # the other positions are left alone
        assert torch.isnan(g[:, :, :i0]).all() and torch.isnan(g[:, :, i0 + ni:]).all()
    h.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_range_with_pairs_context_and_auto_split(precision):
    # a context set to every pair once: the range takes the one-sided fallback
    # (automatic j-split for the range) and agrees with the pairs evaluation
    # to rounding
    n = 4096
    w = disc16k(n)
    path = _kepler_path(w)
    h, st = _ctx(8, w, path, precision, (1, 0, 2, 4))
    h.force_derivs(st)
    full = st.eval.cpu().numpy()
    tol = 1e-13 if precision == "fp64" else 2e-5
    for i0, ni in [(0, 512), (1000, 77), (n - 300, 300)]:
        st.eval.zero_()
        h.force_derivs_range(st, i0, ni)
        g = st.eval.cpu().numpy()
        for k in range(4):
            scale = np.abs(full[k]).max()
            assert np.abs(g[k][:, i0:i0 + ni] - full[k][:, i0:i0 + ni]).max() <= tol * scale, (k, i0, ni)
    h.close()


def test_range_rejects_bad_ranges():
    w = disc16k(100)
    h, st = _ctx(8, w, _kepler_path(w), "fp64", (1, 0, 0, 4))
    for i0, ni in [(-1, 5), (0, 101), (99, 2), (5, -1)]:
        with pytest.raises(HermiteError):
            h.force_derivs_range(st, i0, ni)
    h.force_derivs_range(st, 100, 0)   # an empty range at the end is allowed
    h.close()


@pytest.fixture(scope="module")
def big_disc():
    return large_disc()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_per_gpu_shape_of_the_large_disc(big_disc, precision):
    # one GPU's share of an 8-way division by i of the 1048576-body disc:
    # 131072 i-particles (the fifth eighth) against all j, 8th order; sampled
    # i against the oracle
    w = big_disc
    n = len(w["mass"])
    i0, ni = 4 * (n // 8), n // 8
    _say("per-GPU shape %d x %d %s" % (ni, n, precision))
    path = _kepler_path(w)
    launch = (2, 0, 0, 4) if precision == "fp64" else (1, 0, 1, 4)
    h, st = _ctx(8, w, path, precision, launch)
    h.force_derivs_range(st, i0, ni)
    rng = np.random.default_rng(9)
    il = np.sort(rng.choice(np.arange(i0, i0 + ni), 48, replace=False))
    il[0], il[-1] = i0, i0 + ni - 1
    g = st.eval.cpu().numpy()[:, :, il]
    h.close()
    o, mag, nat = ho.pair_derivs(w["mass"], path, K=3, i_list=il, with_mag=True, with_scale=True)
    if precision == "fp64":
        err = deriv_error(g, o, mag)
        assert within(err, TOL_FP64), err.max(axis=1)
    else:
        err = deriv_error(g, o, mag, nat)
        assert within(err, TOL_MIXED), err.max(axis=1)
    _say("  max err per order", err.max(axis=1))
