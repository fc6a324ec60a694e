"""GPU parity of the O(N^2) evaluation (hermite_force_derivs), the explicit
initial derivatives (hermite_init) and the potential, against the oracle,
element by element, through the C ABI."""
import sys

import numpy as np
import pytest
import torch

from oracle import hermite_oracle as ho
from paper_2006_02501_amd import Hermite
from parity_util import TOL_FP64, TOL_MIXED, deriv_error, disc_path, random_path, within
from workloads import disc16k

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
PAIRS = (1, 0, 2, 4)   # launch shape of the every-pair-once evaluation (j_source 2)


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _eval_gpu(order, mass, path, precision="fp64", eps2=0.0, G=1.0, launch=None):
    p = order // 2 - 1
    n = len(mass)
    h = Hermite(order, max(n, 1), precision=precision, eps2=eps2, G=G, device=DEV)
    st = h.state(mass, path[0], path[1])
    for k in range(p + 1):
        st.pred[k].copy_(torch.as_tensor(np.asarray(path[k], dtype=np.float64).reshape(3, n)))
    if launch is not None:
        h.set_launch(*launch)
    h.force_derivs(st)
    out = st.eval.cpu().numpy()
    h.close()
    return out


@pytest.mark.parametrize("order", [4, 6, 8])
@pytest.mark.parametrize("n", [2, 63, 257, 1000, 2050])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_force_derivs_disc(order, n, precision):
    _say("force_derivs disc order=%d n=%d %s" % (order, n, precision))
    p = order // 2 - 1
    w, path = disc_path(n, p)
    o, mag, nat = ho.pair_derivs(w["mass"], path, K=p, with_mag=True, with_scale=True)
    g = _eval_gpu(order, w["mass"], path, precision)
    err = deriv_error(g, o, mag, None if precision == "fp64" else nat)
    tol = TOL_FP64 if precision == "fp64" else TOL_MIXED
    assert within(err, tol), (err.max(axis=1), tol)


@pytest.mark.parametrize("order", [4, 6, 8])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_force_derivs_random_softened(order, precision):
    _say("force_derivs random softened order=%d %s" % (order, precision))
    rng = np.random.default_rng(order)
    p = order // 2 - 1
    n = 777
    mass, path = random_path(rng, n, p)
    G, eps2 = 0.7, 1e-3
    o, mag, nat = ho.pair_derivs(mass, path, K=p, G=G, eps2=eps2, with_mag=True, with_scale=True)
    g = _eval_gpu(order, mass, path, precision, eps2=eps2, G=G)
    tol = TOL_FP64 if precision == "fp64" else TOL_MIXED
    err = deriv_error(g, o, mag, None if precision == "fp64" else nat)
    assert within(err, tol), (err.max(axis=1), tol)


_SHAPES = [(1, 1, 4), (1, 3, 4), (2, 1, 4), (2, 5, 4), (2, 0, 4), (1, 64, 4), (1, 1, 16), (1, 3, 16),
           (1, 0, 16), (3, 3, 4), (3, 0, 4), (4, 1, 4), (4, 7, 4)]
# 16-wave workgroups and 3-4 i per lane exist only with the scalar j-source
_LAUNCHES = [(sh, src) for sh in _SHAPES for src in (0, 1) if src == 1 or (sh[2] == 4 and sh[0] <= 2)]


@pytest.mark.parametrize("shape,source", _LAUNCHES)
@pytest.mark.parametrize("order", [4, 6, 8])
def test_force_derivs_launch_shapes(order, shape, source):
    # (i_per_thread, j_split, wg_waves) x j_source on a ragged N that spans
    # several tiles, splits and workgroups
    _say("force_derivs launch shape", order, shape, source)
    p = order // 2 - 1
    w, path = disc_path(1500, p)
    o, mag, nat = ho.pair_derivs(w["mass"], path, K=p, with_mag=True, with_scale=True)
    launch = (shape[0], shape[1], source, shape[2])
    g = _eval_gpu(order, w["mass"], path, "fp64", launch=launch)
    assert deriv_error(g, o, mag).max() <= TOL_FP64
    g = _eval_gpu(order, w["mass"], path, "mixed", launch=launch)
    assert within(deriv_error(g, o, mag, nat), TOL_MIXED)


def _pairs_ok(g, o, mag, nat, precision):
    if precision == "fp64":
        return deriv_error(g, o, mag).max() <= TOL_FP64
    if precision == "mixed":
        return within(deriv_error(g, o, mag, nat), TOL_MIXED)
    # split: a, adot at the FP64 bar, the FP32 orders at the mixed bars
    e64 = deriv_error(g[:2], o[:2], mag[:2])
    ok = e64.max() <= TOL_FP64
    if len(g) > 2:
        e32 = deriv_error(g, o, mag, nat)[2:]
        ok = ok and bool(np.all(e32.max(axis=1) <= np.asarray(TOL_MIXED)[2:len(g)]))
    return ok


@pytest.mark.parametrize("precision", ["fp64", "mixed", "split"])
@pytest.mark.parametrize("order", [4, 6, 8])
@pytest.mark.parametrize("n", [2, 3, 63, 64, 65, 255, 256, 257, 511, 700, 1000, 2050])
def test_force_derivs_pairs_once(order, n, precision):
    # every pair taken once for both bodies: ragged n over one and several
    # 256-body super-blocks (diagonal and off-diagonal items, partial blocks)
    _say("force_derivs pairs-once order=%d n=%d %s" % (order, n, precision))
    p = order // 2 - 1
    w, path = disc_path(n, p)
    o, mag, nat = ho.pair_derivs(w["mass"], path, K=p, with_mag=True, with_scale=True)
    g = _eval_gpu(order, w["mass"], path, precision, launch=PAIRS)
    assert _pairs_ok(g, o, mag, nat, precision)


@pytest.mark.parametrize("precision", ["fp64", "mixed", "split"])
@pytest.mark.parametrize("order", [4, 6, 8])
def test_force_derivs_pairs_once_softened_and_reproducible(order, precision):
    _say("force_derivs pairs-once softened order=%d %s" % (order, precision))
    rng = np.random.default_rng(10 + order)
    p = order // 2 - 1
    n = 1531
    mass, path = random_path(rng, n, p)
    o, mag, nat = ho.pair_derivs(mass, path, K=p, eps2=1e-4, G=0.7, with_mag=True, with_scale=True)
    g = _eval_gpu(order, mass, path, precision, eps2=1e-4, G=0.7, launch=PAIRS)
    assert _pairs_ok(g, o, mag, nat, precision)
    assert np.array_equal(g, _eval_gpu(order, mass, path, precision, eps2=1e-4, G=0.7, launch=PAIRS))


@pytest.mark.parametrize("order", [6, 8])
def test_pairs_once_split_low_orders_bitwise_fp64(order):
    # split a and adot take exactly the FP64 pairs kernel's operations
    _say("pairs-once split vs fp64 bitwise order=%d" % order)
    p = order // 2 - 1
    w, path = disc_path(1300, p)
    gs = _eval_gpu(order, w["mass"], path, "split", launch=PAIRS)
    gf = _eval_gpu(order, w["mass"], path, "fp64", launch=PAIRS)
    assert np.array_equal(gs[:2], gf[:2])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_force_derivs_pairs_once_largest(precision):
    # the largest n the every-pair-once path takes (8256 super-block pairs,
    # 406 MB of partials at 8th order), 128 sampled i against the oracle; the
    # path's a and adot are the central body's Kepler field
    _say("pairs-once n=32768", precision)
    n = 32768
    w = disc16k(n)
    x, v = w["x"], w["v"]
    r2 = np.sum(x * x, axis=0)
    rv = np.sum(x * v, axis=0)
    path = [x, v, -x * r2 ** -1.5, -v * r2 ** -1.5 + 3.0 * x * rv * r2 ** -2.5]
    path[2][:, 0] = 0.0
    path[3][:, 0] = 0.0
    rng = np.random.default_rng(12)
    il = np.sort(rng.choice(n, 128, replace=False))
    il[0], il[-1] = 0, n - 1
    o, mag, nat = ho.pair_derivs(w["mass"], path, K=3, i_list=il, with_mag=True, with_scale=True)
    g = _eval_gpu(8, w["mass"], path, precision, launch=PAIRS)[:, :, il]
    if precision == "fp64":
        assert deriv_error(g, o, mag).max() <= TOL_FP64
    else:
        assert within(deriv_error(g, o, mag, nat), TOL_MIXED)


@pytest.mark.parametrize("n", [300, 9217])
@pytest.mark.parametrize("precision", ["fp64", "mixed", "split"])
def test_pairs_once_masked_lanes_stay_finite(precision, n):
    # Bodies 1e4 apart whose path adot is ~1e33: every real pair's chain fits
    # FP32 (it is scaled by 1/r^2 ~ 1e-8), but a lane that must drop its pair
    # (the second half of the diagonal block's step 32, or a padding body of
    # the ragged last super-block) would overflow FP32 at w = 1 and put
    # 0 * inf = NaN into real sums.  Such lanes take a zero path instead.
    # n = 300: a full super-block and a ragged one, one workgroup per item
    # and phase; n = 9217: one workgroup per item, a last super-block of one
    # body (sampled i against the oracle).
    _say("pairs-once masked lanes n=%d %s" % (n, precision))
    rng = np.random.default_rng(21)
    mass = rng.uniform(0.5, 1.5, n)
    path = [rng.uniform(-1e4, 1e4, (3, n)), rng.normal(size=(3, n)) * 1e3,
            rng.normal(size=(3, n)) * 1e10, rng.normal(size=(3, n)) * 1e33]
    il = None
    if n > 1000:
        il = np.sort(rng.choice(n, 64, replace=False))
        il[0], il[-1] = 0, n - 1
    o, mag, nat = ho.pair_derivs(mass, path, K=3, i_list=il, with_mag=True, with_scale=True)
    g = _eval_gpu(8, mass, path, precision, launch=PAIRS)
    assert np.all(np.isfinite(g))
    if il is not None:
        g = g[:, :, il]
    assert _pairs_ok(g, o, mag, nat, precision)


def test_pairs_once_limits():
    _say("pairs-once limits")
    from paper_2006_02501_amd import HermiteError
    h = Hermite(8, 16, device=DEV)
    for bad in [(2, 0, 2, 4), (1, 0, 2, 16)]:
        with pytest.raises(HermiteError):
            h.set_launch(*bad)
    h.close()


def _kepler_path(w, K):
    # the central body's Kepler field as the path's a and adot
    x, v = w["x"], w["v"]
    r2 = np.sum(x * x, axis=0)
    rv = np.sum(x * v, axis=0)
    path = [x, v, -x * r2 ** -1.5, -v * r2 ** -1.5 + 3.0 * x * rv * r2 ** -2.5]
    path[2][:, 0] = 0.0
    path[3][:, 0] = 0.0
    return path[:K + 1]


@pytest.mark.parametrize("order", [4, 8])
@pytest.mark.parametrize("precision", ["fp64", "mixed", "split"])
def test_force_derivs_pairs_once_whole_items_ragged(order, precision):
    # Launches of few items take one workgroup per item and phase (every n
    # the tests above use); from ~6900 bodies (~9000 at 4th order) on, one
    # workgroup per item.  n = 9217: 703 items, whole on this GPU at every
    # order, with a last super-block of one body.  Sampled i (the ragged
    # block's body among them) against the oracle.
    _say("pairs-once whole items n=9217 order=%d %s" % (order, precision))
    n = 9217
    p = order // 2 - 1
    w = disc16k(n)
    path = _kepler_path(w, p)
    rng = np.random.default_rng(13)
    il = np.sort(rng.choice(n, 96, replace=False))
    il[0], il[-1] = 0, n - 1
    o, mag, nat = ho.pair_derivs(w["mass"], path, K=p, i_list=il, with_mag=True, with_scale=True)
    g = _eval_gpu(order, w["mass"], path, precision, launch=PAIRS)[:, :, il]
    assert _pairs_ok(g, o, mag, nat, precision)


@pytest.mark.parametrize("order,n", [(4, 32769), (8, 40000), (6, 50000)])
@pytest.mark.parametrize("precision", ["fp64", "mixed", "split"])
def test_force_derivs_pairs_once_chunked(order, n, precision):
    # beyond 32768 bodies: chunks of up to 64 super-blocks, one launch per
    # chunk pair (triangles and rectangles, a last chunk of 1 super-block at
    # n = 32769 and partial ones otherwise); sampled i against the oracle,
    # and the FP64 result against the LDS kernel's
    _say("pairs-once chunked order=%d n=%d %s" % (order, n, precision))
    p = order // 2 - 1
    w = disc16k(n)
    path = _kepler_path(w, p)
    rng = np.random.default_rng(n)
    il = np.sort(rng.choice(n, 160, replace=False))
    il[0], il[-1] = 0, n - 1
    o, mag, nat = ho.pair_derivs(w["mass"], path, K=p, i_list=il, with_mag=True, with_scale=True)
    g = _eval_gpu(order, w["mass"], path, precision, launch=PAIRS)
    assert _pairs_ok(g[:, :, il], o, mag, nat, precision)
    if precision == "fp64":
        ref = _eval_gpu(order, w["mass"], path, "fp64", launch=(2, 4, 0, 4))
        scale = np.abs(ref).max(axis=(1, 2), keepdims=True)
        assert (np.abs(g - ref) / scale).max() <= 1e-13
        assert np.array_equal(g, _eval_gpu(order, w["mass"], path, precision, launch=PAIRS))


def test_set_launch_validation():
    h = Hermite(8, 16, device=DEV)
    from paper_2006_02501_amd import HermiteError
    for bad in [(5, 0, 1, 4), (0, 0, 1, 4), (3, 0, 0, 4), (4, 0, 1, 16), (1, 65, 1, 4), (1, 0, 3, 4),
                (1, 0, 1, 8), (2, 0, 1, 16), (1, 0, 0, 16)]:
        with pytest.raises(HermiteError):
            h.set_launch(*bad)
    h.set_launch(1, 0, 1, 16)
    h.close()


@pytest.mark.parametrize("launch", [None, PAIRS])
def test_force_derivs_single_particle_and_empty(launch):
    _say("force_derivs n=1 and n=0", launch)
    for prec in ("fp64", "mixed", "split"):
        g = _eval_gpu(8, np.array([1.0]), [np.ones((3, 1))] * 4, prec, launch=launch)
        assert np.array_equal(g, np.zeros((4, 3, 1)))
    h = Hermite(8, 0, device=DEV)
    if launch is not None:
        h.set_launch(*launch)
    st = h.state(np.zeros(0), np.zeros((3, 0)), np.zeros((3, 0)))
    h.force_derivs(st)
    h.init(st)
    h.step(st, 0.1, 2)
    h.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed", "split"])
def test_force_derivs_pairs_once_coincident_softened(precision):
    # bodies at the same place with softening: the pair terms are finite
    # (r = 0 gives zero force, the softened derivatives stay finite)
    _say("pairs-once coincident softened", precision)
    n = 300
    rng = np.random.default_rng(8)
    mass, path = random_path(rng, n, 3)
    for k in range(4):
        path[k][:, 100:110] = path[k][:, 100:101]      # ten bodies at one point with one path
    o, mag, nat = ho.pair_derivs(mass, path, K=3, eps2=1e-6, with_mag=True, with_scale=True)
    g = _eval_gpu(8, mass, path, precision, eps2=1e-6, launch=PAIRS)
    assert np.all(np.isfinite(g))
    assert _pairs_ok(g, o, mag, nat, precision)


def test_force_derivs_bitwise_reproducible():
    _say("force_derivs reproducibility")
    w, path = disc_path(3000, 3)
    a = _eval_gpu(8, w["mass"], path, "fp64")
    b = _eval_gpu(8, w["mass"], path, "fp64")
    assert np.array_equal(a, b)
    c = _eval_gpu(8, w["mass"], path, "mixed")
    d = _eval_gpu(8, w["mass"], path, "mixed")
    assert np.array_equal(c, d)


# Launch shapes (i_per_thread, j_split, j_source, wg_waves) checked at the
# full 16k size: every pair once (what the benchmark's autotuner picks on
# this disc for all three chains, and what its traffic profile was taken
# with), the scalar stream with 64 splits and the LDS tiles with 4 splits
# (the earlier picks).
FULL_SIZE_SHAPES = [PAIRS, (1, 64, 1, 4), (2, 4, 0, 4)]


def _eval_autotuned(order, mass, path, precision):
    p = order // 2 - 1
    n = len(mass)
    h = Hermite(order, n, precision=precision, device=DEV)
    st = h.state(mass, path[0], path[1])
    for k in range(p + 1):
        st.pred[k].copy_(torch.as_tensor(np.asarray(path[k], dtype=np.float64).reshape(3, n)))
    shape = h.autotune(st)
    h.force_derivs(st)
    out = st.eval.cpu().numpy()
    h.close()
    return out, shape


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_force_derivs_full_size_sampled(precision):
    # Disc of 16384 bodies (8th order): the default launch, the shapes above
    # (the first is the one the benchmark times) and whatever the autotuner
    # picks on this device; 512 sampled i-particles checked against the
    # oracle, and (FP64) the runs against each other.
    _say("force_derivs N=16384 sampled", precision)
    n = 16384
    w, path = disc_path(n, 3)
    rng = np.random.default_rng(99)
    il = np.sort(rng.choice(n, 512, replace=False))
    il[0] = 0                     # the central body
    o, mag, nat = ho.pair_derivs(w["mass"], path, K=3, i_list=il, with_mag=True, with_scale=True)
    tol = TOL_FP64 if precision == "fp64" else TOL_MIXED
    runs = [("default", _eval_gpu(8, w["mass"], path, precision))]
    for shape in FULL_SIZE_SHAPES:
        runs.append((str(shape), _eval_gpu(8, w["mass"], path, precision, launch=shape)))
    g_tuned, shape = _eval_autotuned(8, w["mass"], path, precision)
    runs.append(("autotuned %s" % (shape,), g_tuned))
    for name, g in runs:
        err = deriv_error(g[:, :, il], o, mag, None if precision == "fp64" else nat)
        _say("  %s %s max err per order %s" % (precision, name, err.max(axis=1)))
        assert within(err, tol), (precision, name, err.max(axis=1))
    if precision == "fp64":
        # every launch shape sums the same FP64 terms; they differ only in
        # the order of the additions
        ref = runs[1][1]
        scale = np.abs(ref).max(axis=(1, 2), keepdims=True)
        for _, g in runs:
            assert (np.abs(g - ref) / scale).max() <= 1e-13


@pytest.mark.parametrize("order", [4, 6, 8])
def test_init_parity(order):
    _say("init order=%d" % order)
    p = order // 2 - 1
    w = disc_path(900, 1)[0]
    st_o = ho.State(w["mass"], w["x"], w["v"], p)
    ho.init_derivs(st_o, eps2=1e-6)
    h = Hermite(order, 900, eps2=1e-6, device=DEV)
    st = h.state(w["mass"], w["x"], w["v"])
    h.init(st)
    g = st.deriv.cpu().numpy()
    assert st.initialized
    for k in range(2 * p):
        o = st_o.derivs[k]
        # per-particle relative error of the derivative vector
        num = np.abs(g[k] - o).max(axis=0)
        den = np.sqrt((o * o).sum(axis=0))
        assert (num / den).max() <= 1e-11, (k, (num / den).max())
    h.close()


def test_potential_parity():
    _say("potential")
    w, _ = disc_path(1234, 1)
    h = Hermite(4, 1234, eps2=1e-5, device=DEV)
    st = h.state(w["mass"], w["x"], w["v"])
    phi = h.potential(st).cpu().numpy()
    o = ho.potential_per_particle(w["mass"], w["x"], eps2=1e-5)
    assert np.abs(phi - o).max() <= 1e-13 * np.abs(o).max()
    h.close()
