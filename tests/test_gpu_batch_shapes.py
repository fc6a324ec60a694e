"""Launch shapes of the batched form (hermite_batch_set_launch / autotune):
every shape against the oracle on bins that take every sweep and its edges,
the full 4096-system workload checked system by system (bitwise across
persistent grids, against per-system hermite_step runs), and the autotuner's
cache."""
import sys

import numpy as np
import pytest
import torch

from oracle import hermite_oracle as ho
from paper_2006_02501_amd import BatchHermite, Hermite, HermiteError, tune_cache_clear
from parity_util import rel_max
from workloads import batch_systems

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# (waves, ring_min): one, two and four waves per bin; the whole-wave ring
# from 57 bodies, or per-system rings only
SHAPES = [(1, 57), (2, 57), (4, 57), (1, 65), (2, 65), (4, 65)]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def batch_workload():
    return batch_systems()


def _edge_set(wb, want):
    offs = wb["offsets"]
    sizes = np.diff(offs)
    mass, xs, vs, dts = [], [], [], []
    for n in want:
        s = int(np.nonzero(sizes == max(n, 3))[0][0])
        lo = offs[s]
        mass.append(wb["mass"][lo:lo + n])
        xs.append(wb["x"][:, lo:lo + n])
        vs.append(wb["v"][:, lo:lo + n])
        dts.append(wb["dt"][s])
    off = np.concatenate([[0], np.cumsum(want)]).astype(np.int64)
    return dict(offsets=off, mass=np.concatenate(mass), x=np.ascontiguousarray(np.concatenate(xs, axis=1)),
                v=np.ascontiguousarray(np.concatenate(vs, axis=1)), dt=np.array(dts))


# Sizes whose first-fit-decreasing bins take both sweeps and their edges:
# whole-wave rings (64; 58 + 6; 57 + 7), per-system rings (56 + 8; 48 + 16;
# 33 + 31, even sizes with a half last step; 7 + 3 + 2 + 1, with a two-body
# and a one-body system).  At 4th and 6th order a shorter set.
EDGE = {8: [64, 58, 6, 57, 7, 56, 8, 48, 16, 33, 31, 7, 3, 2, 1], 6: [64, 58, 6, 56, 8, 5], 4: [64, 58, 6, 56, 8, 5]}
STEPS = 10


@pytest.fixture(scope="module")
def oracle_edges(batch_workload):
    """Oracle states after STEPS P(EC)^3 steps of every edge set, per order."""
    out = {}
    for order, want in EDGE.items():
        e = _edge_set(batch_workload, want)
        p = order // 2 - 1
        res = []
        for k in range(len(want)):
            lo, hi = e["offsets"][k], e["offsets"][k + 1]
            o = ho.State(e["mass"][lo:hi], e["x"][:, lo:hi], e["v"][:, lo:hi], p)
            ho.init_derivs(o)
            for _ in range(STEPS):
                ho.step(o, e["dt"][k], 3)
            res.append((o.x.copy(), o.v.copy()))
        out[order] = (e, res)
    return out


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("order", [8, 6, 4])
def test_shapes_match_oracle(oracle_edges, order, precision, shape):
    _say("batch shape %s order=%d %s" % (shape, order, precision))
    e, res = oracle_edges[order]
    bh = BatchHermite(order, e["offsets"], precision=precision, device=DEV)
    bh.set_launch(0, *shape)
    assert bh.get_launch()[1:] == shape
    st = bh.state(e["mass"], e["x"], e["v"])
    bh.init(st)
    bh.run(st, e["dt"], STEPS, 3)
    d = st.host()
    bh.close()
    tol = 1e-11 if precision == "fp64" else 1e-6
    for k, (ox, ov) in enumerate(res):
        lo, hi = e["offsets"][k], e["offsets"][k + 1]
        assert np.all(np.isfinite(d["x"][:, lo:hi])), k
        assert rel_max(d["x"][:, lo:hi], ox) <= tol, (k, hi - lo)
        assert rel_max(d["v"][:, lo:hi], ov) <= tol * 10, (k, hi - lo)


@pytest.mark.parametrize("shape", [(4, 57), (2, 57), (1, 65)])
def test_shapes_compensated_match_oracle(batch_workload, shape):
    # compensated summation (Sec. 3.2) in the multi-wave and LDS-sum kernels:
    # against the oracle's compensated steps
    _say("batch shape %s compensated" % (shape,))
    e = _edge_set(batch_workload, [60, 4, 33, 31])
    bh = BatchHermite(8, e["offsets"], device=DEV, compensated=True)
    bh.set_launch(0, *shape)
    st = bh.state(e["mass"], e["x"], e["v"])
    bh.init(st)
    steps = 30
    bh.run(st, e["dt"], steps, 3)
    d = st.host()
    bh.close()
    for k in range(4):
        lo, hi = e["offsets"][k], e["offsets"][k + 1]
        o = ho.State(e["mass"][lo:hi], e["x"][:, lo:hi], e["v"][:, lo:hi], 3)
        ho.init_derivs(o)
        for _ in range(steps):
            ho.step(o, e["dt"][k], 3, compensated=True)
        assert rel_max(d["x"][:, lo:hi], o.x) <= 1e-11, k
        assert rel_max(d["v"][:, lo:hi], o.v) <= 1e-10, k


@pytest.mark.parametrize("shape", [(4, 57), (2, 57), (1, 57), (4, 65)])
def test_shapes_per_system_iterations(batch_workload, shape):
    # per-system iteration counts: each system bitwise as a run with its own n
    # everywhere (same shape, same bins)
    _say("batch shape %s per-system n" % (shape,))
    e = _edge_set(batch_workload, [60, 4, 33, 31, 7, 3])
    iters = np.array([1, 2, 3, 4, 2, 3], dtype=np.int32)
    bh = BatchHermite(8, e["offsets"], device=DEV)
    bh.set_launch(0, *shape)
    st = bh.state(e["mass"], e["x"], e["v"])
    bh.init(st)
    bh.run(st, e["dt"], 12, iters)
    d = st.host()
    for n in (1, 2, 3, 4):
        u = bh.state(e["mass"], e["x"], e["v"])
        bh.init(u)
        bh.run(u, e["dt"], 12, n)
        du = u.host()
        for k in np.nonzero(iters == n)[0]:
            lo, hi = e["offsets"][k], e["offsets"][k + 1]
            assert np.array_equal(d["x"][:, lo:hi], du["x"][:, lo:hi]), (k, n)
            assert np.array_equal(d["v"][:, lo:hi], du["v"][:, lo:hi]), (k, n)
    bh.close()


def _run_full(wb, precision, shape, workgroups, steps):
    bh = BatchHermite(8, wb["offsets"], precision=precision, device=DEV)
    bh.set_launch(workgroups, *shape)
    st = bh.state(wb["mass"], wb["x"], wb["v"])
    bh.init(st)
    bh.run(st, wb["dt"], steps, wb["n_iter"])
    d = st.host()
    used = bh.get_launch()
    bh.close()
    return d, used


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_every_system(batch_workload, precision):
    """All 4096 systems (2156 bins), each one checked:
    - bitwise the same with the full persistent grid and with 61 workgroups
      (a bin is computed by one workgroup in a fixed order whatever the grid,
      so a skipped, doubled or misassigned bin shows up as a difference),
      for two, four and one waves per bin;
    - finite and moved from its start;
    - against hermite_step run on that system alone: within 1e-12 (FP64) of
      the largest |x| and |v| of the system, or the mixed step bound (mixed,
      against the FP64 single-system run)."""
    wb = batch_workload
    offs = wb["offsets"]
    steps = 3
    _say("batch full size every system %s" % precision)
    base = {}
    for shape in [(2, 57), (4, 57), (1, 57)]:
        d_full, used = _run_full(wb, precision, shape, 0, steps)
        d_61, used61 = _run_full(wb, precision, shape, 61, steps)
        assert used61[0] == 61 and used[0] > 61
        _say("  shape %s: grids %d and %d" % (shape, used[0], used61[0]))
        for key in ("x", "v"):
            diff = np.nonzero(np.any(d_full[key] != d_61[key], axis=0))[0]
            assert diff.size == 0, ("bodies differ between grids", shape, key, diff[:10])
        assert all(np.array_equal(p, q) for p, q in zip(d_full["derivs"], d_61["derivs"]))
        base[shape] = d_full
    d = base[(2, 57)]
    assert np.all(np.isfinite(d["x"])) and np.all(np.isfinite(d["v"]))
    moved = np.any(d["x"] != wb["x"], axis=0)
    assert moved.all(), np.nonzero(~moved)[0][:10]
    # every system alone through hermite_step (one context reused)
    h = Hermite(8, 64, device=DEV)
    worst = 0.0
    tol = 1e-12 if precision == "fp64" else 1e-6
    for s in range(len(offs) - 1):
        lo, hi = offs[s], offs[s + 1]
        st = h.state(wb["mass"][lo:hi], wb["x"][:, lo:hi], wb["v"][:, lo:hi])
        h.init(st)
        for _ in range(steps):
            h.step(st, wb["dt"][s], wb["n_iter"])
        g = st.host()
        ex = rel_max(d["x"][:, lo:hi], g["x"])
        ev = rel_max(d["v"][:, lo:hi], g["v"])
        worst = max(worst, ex, ev)
        assert ex <= tol and ev <= tol * 10, (s, hi - lo, ex, ev)
    h.close()
    _say("  worst difference from per-system runs: %.2e" % worst)


def test_autotune_cache_and_state(batch_workload):
    """The batched autotuner leaves the state alone, picks a valid shape,
    caches it (a second call times nothing), and a run with the picked shape
    is bitwise the run with that shape set by hand."""
    wb = batch_workload
    rng = np.random.default_rng(11)
    systems = np.sort(rng.choice(len(wb["dt"]), 300, replace=False))
    offs = wb["offsets"]
    idx = np.concatenate([np.arange(offs[s], offs[s + 1]) for s in systems])
    sizes = [offs[s + 1] - offs[s] for s in systems]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    mass, x, v, dt = wb["mass"][idx], wb["x"][:, idx], wb["v"][:, idx], wb["dt"][systems]
    tune_cache_clear()
    bh = BatchHermite(8, off, device=DEV)
    st = bh.state(mass, x, v)
    bh.init(st)
    before = st.host()
    shape, cached = bh.autotune(st, dt, 4, 3)
    after = st.host()
    assert not cached
    assert np.array_equal(before["x"], after["x"]) and np.array_equal(before["v"], after["v"])
    assert all(np.array_equal(p, q) for p, q in zip(before["derivs"], after["derivs"]))
    wg, waves, ring_min = shape
    assert 1 <= wg and waves in (1, 2, 4) and 2 <= ring_min <= 65
    assert bh.get_launch() == shape
    bh.run(st, dt, 6, 3)
    a = st.host()
    bh.close()
    bh2 = BatchHermite(8, off, device=DEV)
    st2 = bh2.state(mass, x, v)
    bh2.init(st2)
    shape2, cached2 = bh2.autotune(st2, dt, 4, 3)
    assert cached2 and shape2 == shape
    bh2.set_launch(*shape)
    bh2.run(st2, dt, 6, 3)
    b = st2.host()
    bh2.close()
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["v"], b["v"])
    tune_cache_clear()
    bh3 = BatchHermite(8, off, device=DEV)
    st3 = bh3.state(mass, x, v)
    bh3.init(st3)
    _, cached3 = bh3.autotune(st3, dt, 4, 3)
    assert not cached3
    bh3.close()


def test_set_launch_rejects_bad_shapes(batch_workload):
    e = _edge_set(batch_workload, [10, 5])
    bh = BatchHermite(8, e["offsets"], device=DEV)
    for bad in [(-1, 4, 57), (0, 3, 57), (0, 8, 57), (0, 4, 1), (0, 4, 66)]:
        with pytest.raises(HermiteError):
            bh.set_launch(*bad)
    h = Hermite(8, 16, device=DEV)
    assert h.lib.hermite_batch_set_launch(h.ctx, 0, 4, 57) == -1   # not a batched context
    h.close()
    bh.close()


def test_graph_recaptured_on_shape_change(batch_workload):
    # the captured graph is keyed by the launch shape: a new shape re-captures,
    # and a new grid gives the same bits
    e = _edge_set(batch_workload, [64, 58, 6, 33, 31])
    bh = BatchHermite(8, e["offsets"], device=DEV)
    a = bh.state(e["mass"], e["x"], e["v"])
    bh.init(a)
    b = bh.state(e["mass"], e["x"], e["v"])
    bh.init(b)
    dt = torch.as_tensor(e["dt"]).to(DEV)
    bh.set_launch(0, 4, 57)
    bh.run(a, dt, 8, 3)
    bh.set_launch(1, 4, 57)
    bh.run(b, dt, 8, 3)
    da, db = a.host(), b.host()
    assert np.array_equal(da["x"], db["x"]) and np.array_equal(da["v"], db["v"])
    bh.close()


def test_default_shape_follows_the_batch(batch_workload):
    # one wave when no system has more than 16 bodies; four when every bin
    # fits on the GPU at once with four waves (a few bins); two for the full
    # workload (2156 bins, more than the GPU holds at four waves each)
    cases = [([64], 4), ([64, 58, 6, 33, 31], 4), ([2, 2, 2], 1), ([16, 16, 9], 1)]
    for sizes, waves in cases:
        e = _edge_set(batch_workload, sizes)
        for precision in ("fp64", "mixed"):
            bh = BatchHermite(8, e["offsets"], precision=precision, device=DEV)
            wg, w, rm = bh.get_launch()
            assert (w, rm) == (waves, 57), (sizes, precision, wg, w, rm)
            assert 1 <= wg <= len(sizes)
            bh.close()
    bh = BatchHermite(8, batch_workload["offsets"], device=DEV)
    assert bh.get_launch()[1:] == (2, 57)
    bh.close()
