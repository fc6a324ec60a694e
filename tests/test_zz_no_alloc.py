"""hermite_force_derivs_noalloc (the evaluation without a context, for callers
that cannot allocate) against hermite_force_derivs on the same inputs: two
calls in a row, the second with fewer bodies, in every chain; device memory
unchanged by a call; argument errors; replays of a captured graph."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_2006_02501_amd import Hermite, HermiteError, force_derivs_noalloc, load_library
from paper_2006_02501_amd.hermite import Params, StateC
from workloads import disc16k

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _state(order, n, precision):
    """A disc of n bodies with a realistic path (x, v, a, adot from the GPU's
    initialisation) in st.pred, and the context's own evaluation of it."""
    w = disc16k(n)
    h = Hermite(order, n, precision=precision, device=DEV)
    st = h.state(w["mass"], w["x"], w["v"])
    h.init(st)
    p = order // 2 - 1
    st.pred[0].copy_(st.pos)
    st.pred[1].copy_(st.vel)
    for k in range(p - 1):
        st.pred[2 + k].copy_(st.deriv[k])
    h.set_launch(1, 0, 2, 4)   # every pair once, as the no-alloc call computes it
    h.force_derivs(st)
    ref = st.eval.clone()
    st.eval.zero_()
    return h, st, ref


def _rel_per_order(g, o):
    g = g.cpu().numpy()
    o = o.cpu().numpy()
    return [float(np.abs(g[k] - o[k]).max() / np.abs(o[k]).max()) for k in range(o.shape[0])]


@pytest.mark.parametrize("order,precision", [(8, "fp64"), (8, "mixed"), (8, "split"), (6, "fp64"), (4, "fp64")])
def test_noalloc_matches_context_two_calls(order, precision):
    # first call: 16384 bodies (at 8th order more than one launch holds: pairs
    # of chunks); second call: 3000 bodies (one launch, split by phase)
    cases = [(16384, 1e-13), (3000, 1e-13)]
    prepared = [(_state(order, n, precision), tol, n) for n, tol in cases]
    torch.cuda.synchronize()
    for call, ((h, st, ref), tol, n) in enumerate(prepared):
        _say("noalloc order=%d %s n=%d" % (order, precision, n))
        free_before = torch.cuda.mem_get_info(0)[0]
        force_derivs_noalloc(order, st, precision=precision, device=DEV)
        torch.cuda.synchronize()
        if call > 0:
            # a call after the first on this device allocates nothing
            assert torch.cuda.mem_get_info(0)[0] == free_before
        assert torch.isfinite(st.eval).all()
        err = _rel_per_order(st.eval, ref)
        _say("  max diff per order vs hermite_force_derivs: %s" % ", ".join("%.1e" % e for e in err))
        assert max(err) <= tol, err
        h.close()


def test_noalloc_argument_errors():
    lib = load_library()
    w = disc16k(100)
    h = Hermite(8, 100, device=DEV)
    st = h.state(w["mass"], w["x"], w["v"])
    bad = Params(5, 0, 0, 0, 1.0, 0.0, 0, 0)
    assert lib.hermite_force_derivs_noalloc(ctypes.byref(bad), ctypes.byref(st.c), None) == -2
    assert b"order" in lib.hermite_last_error(None)
    good = Params(8, 0, 0, 0, 1.0, 0.0, 0, 0)
    assert lib.hermite_force_derivs_noalloc(ctypes.byref(good), None, None) == -1
    big = StateC()
    big.n = (1 << 40) + 1
    assert lib.hermite_force_derivs_noalloc(ctypes.byref(good), ctypes.byref(big), None) == -1
    assert b"n outside" in lib.hermite_last_error(None)
    neg = Params(8, 0, 0, 0, 1.0, -1.0, 0, 0)
    assert lib.hermite_force_derivs_noalloc(ctypes.byref(neg), ctypes.byref(st.c), None) == -1
    with pytest.raises(HermiteError):
        force_derivs_noalloc(8, st, precision="fp64", eps2=-1.0, device=DEV)
    h.close()


def test_noalloc_graph_replays():
    # captured into a HIP graph (through torch's capture of its current
    # stream) and replayed three times, with eager work in between; every
    # replay equals the eager result bitwise
    h, st, ref = _state(8, 2000, "fp64")
    force_derivs_noalloc(8, st, device=DEV)   # first call on the device outside the capture
    torch.cuda.synchronize()
    eager = st.eval.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            force_derivs_noalloc(8, st, device=DEV)
    torch.cuda.synchronize()
    for r in range(3):
        st.eval.fill_(float(r + 1))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(st.eval, eager), r
        _ = (st.pos * 2.0).sum().item()   # unrelated eager work between replays
    assert max(_rel_per_order(eager, ref)) <= 1e-13
    h.close()
