"""Python binding of ``libhermite.so`` -- argument marshalling only.

Every step of the method runs in the library's HIP kernels; PyTorch only
provides device memory (FP64 tensors, structure-of-arrays) and the HIP stream.
If the library has not been built this module raises on first use: there is
no CPU fallback.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhermite.so")

HERMITE_OK = 0
STATUS = {0: "OK", -1: "E_ARG", -2: "E_ORDER", -3: "E_ALLOC", -4: "E_HIP", -5: "E_NONFINITE", -6: "E_STATE"}
PRECISIONS = {"fp64": 0, "mixed": 1, "split": 2}
CORRECTORS = {"modified": 0, "beta1": 1, "shifted": 2}


class HermiteError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, msg))
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("precision", ctypes.c_int32), ("corrector", ctypes.c_int32),
                ("check_finite", ctypes.c_int32), ("G", ctypes.c_double), ("eps2", ctypes.c_double),
                ("compensated", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class StateC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("mass", ctypes.c_void_p), ("pos", ctypes.c_void_p),
                ("vel", ctypes.c_void_p), ("deriv", ctypes.c_void_p), ("pred", ctypes.c_void_p),
                ("eval", ctypes.c_void_p), ("t", ctypes.c_double), ("initialized", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("comp", ctypes.c_void_p), ("t_comp", ctypes.c_double)]


class VstepCfg(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("t_end", ctypes.c_double), ("rec_from", ctypes.c_double),
                ("n_iter", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class VstepResult(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("E0", ctypes.c_double), ("steps", ctypes.c_int64),
                ("records", ctypes.c_int32), ("failed", ctypes.c_int32), ("rec_overflow", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_lib = None

# name -> (restype, argtypes); mirrors include/hermite.h
_P = ctypes.c_void_p
_SIGS = {
    "hermite_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int64, _P, ctypes.POINTER(_P)]),
    "hermite_destroy": (ctypes.c_int, [_P]),
    "hermite_set_stream": (ctypes.c_int, [_P, _P]),
    "hermite_init": (ctypes.c_int, [_P, ctypes.POINTER(StateC)]),
    "hermite_predict": (ctypes.c_int, [_P, ctypes.POINTER(StateC), ctypes.c_double]),
    "hermite_force_derivs": (ctypes.c_int, [_P, ctypes.POINTER(StateC)]),
    "hermite_force_derivs_range": (ctypes.c_int, [_P, ctypes.POINTER(StateC), ctypes.c_int64, ctypes.c_int64]),
    "hermite_correct": (ctypes.c_int, [_P, ctypes.POINTER(StateC), ctypes.c_double, ctypes.c_int32]),
    "hermite_step": (ctypes.c_int, [_P, ctypes.POINTER(StateC), ctypes.c_double, ctypes.c_int32]),
    "hermite_potential": (ctypes.c_int, [_P, ctypes.POINTER(StateC), _P]),
    "hermite_step_criterion": (ctypes.c_int, [_P, ctypes.POINTER(StateC), ctypes.c_double,
                                              ctypes.POINTER(ctypes.c_double)]),
    "hermite_step_symmetric": (ctypes.c_int, [_P, ctypes.POINTER(StateC), ctypes.c_double, ctypes.c_int32,
                                              ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
    "hermite_batch_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                            _P, ctypes.POINTER(_P)]),
    "hermite_batch_init": (ctypes.c_int, [_P, ctypes.POINTER(StateC)]),
    "hermite_batch_run": (ctypes.c_int, [_P, ctypes.POINTER(StateC), _P, ctypes.c_int32, ctypes.c_int32]),
    "hermite_batch_run_iters": (ctypes.c_int, [_P, ctypes.POINTER(StateC), _P, ctypes.c_int32,
                                               ctypes.POINTER(ctypes.c_int32)]),
    "hermite_ensemble_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int32,
                                               ctypes.POINTER(ctypes.c_int64), _P, ctypes.POINTER(_P)]),
    "hermite_ensemble_init": (ctypes.c_int, [_P, ctypes.POINTER(StateC)]),
    "hermite_ensemble_run": (ctypes.c_int, [_P, ctypes.POINTER(StateC), ctypes.POINTER(VstepCfg), ctypes.c_int64,
                                            ctypes.c_int32, _P, ctypes.POINTER(VstepResult)]),
    "hermite_set_launch": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "hermite_autotune": (ctypes.c_int, [_P, ctypes.POINTER(StateC), ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32)]),
    "hermite_batch_set_launch": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "hermite_batch_get_launch": (ctypes.c_int, [_P] + [ctypes.POINTER(ctypes.c_int32)] * 3),
    "hermite_batch_autotune": (ctypes.c_int, [_P, ctypes.POINTER(StateC), _P, ctypes.c_int32, ctypes.c_int32]
                               + [ctypes.POINTER(ctypes.c_int32)] * 4),
    "hermite_tune_cache_clear": (None, []),
    "hermite_force_derivs_noalloc": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.POINTER(StateC), _P]),
    "hermite_last_error": (ctypes.c_char_p, [_P]),
    "hermite_version": (ctypes.c_char_p, []),
    "hermite_fma_rate": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
}


def load_library():
    """Load libhermite.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libhermite.so is not built (%s); run paper_2006_02501_amd/build.py "
                              "or __graft_entry__.build()" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _check(ctx, status):
    if status != HERMITE_OK:
        msg = load_library().hermite_last_error(ctx)
        raise HermiteError(status, msg.decode() if msg else "")


def _stream_handle(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class DeviceState:
    """Particle state of an order-2(p+1) integrator in device memory (FP64, SoA)."""

    def __init__(self, p, mass, x, v, device, t=0.0, with_pred=True):
        self.p = p
        dev = torch.device(device)
        self.mass = torch.as_tensor(np.ascontiguousarray(mass, dtype=np.float64)).to(dev)
        n = self.mass.shape[0]
        self.pos = torch.as_tensor(np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(3, n))).to(dev)
        self.vel = torch.as_tensor(np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(3, n))).to(dev)
        self.deriv = torch.zeros((2 * p, 3, n), dtype=torch.float64, device=dev)
        if with_pred:
            self.pred = torch.zeros((p + 1, 3, n), dtype=torch.float64, device=dev)
            self.eval = torch.zeros((p + 1, 3, n), dtype=torch.float64, device=dev)
        else:
            self.pred = self.eval = None
        # compensation terms of x and v (used with compensated summation)
        self.comp = torch.zeros((2, 3, n), dtype=torch.float64, device=dev)
        self.c = StateC()
        self.c.n = n
        self.c.mass = self.mass.data_ptr()
        self.c.pos = self.pos.data_ptr()
        self.c.vel = self.vel.data_ptr()
        self.c.deriv = self.deriv.data_ptr()
        self.c.pred = self.pred.data_ptr() if with_pred else None
        self.c.eval = self.eval.data_ptr() if with_pred else None
        self.c.comp = self.comp.data_ptr()
        self.c.t = float(t)
        self.c.t_comp = 0.0
        self.c.initialized = 0

    @property
    def n(self):
        return self.c.n

    @property
    def t(self):
        return self.c.t

    @property
    def initialized(self):
        return bool(self.c.initialized)

    def mark_initialized(self):
        """For a state restored from a checkpoint (t, mass, pos, vel, deriv)."""
        self.c.initialized = 1

    def host(self):
        """Copy the state to the host as numpy arrays (synchronises)."""
        d = dict(mass=self.mass.cpu().numpy(), x=self.pos.cpu().numpy(), v=self.vel.cpu().numpy(),
                 derivs=[q for q in self.deriv.cpu().numpy()], t=self.t)
        if self.pred is not None:
            d["pred"] = [q for q in self.pred.cpu().numpy()]
            d["eval"] = [q for q in self.eval.cpu().numpy()]
        comp = self.comp.cpu().numpy()
        d["cx"], d["cv"], d["t_comp"] = comp[0], comp[1], self.c.t_comp
        return d


class Hermite:
    """One integrator context (hermite_create) bound to a torch device and stream."""

    def __init__(self, order, n_max, precision="fp64", corrector="modified", G=1.0, eps2=0.0,
                 check_finite=False, device="cuda:0", compensated=False):
        self.lib = load_library()
        self.order = order
        self.p = order // 2 - 1
        self.device = torch.device(device)
        self.prm = Params(order, PRECISIONS[precision], CORRECTORS[corrector], 1 if check_finite else 0,
                          float(G), float(eps2), 1 if compensated else 0, 0)
        self.ctx = ctypes.c_void_p()
        _check(None, self.lib.hermite_create(ctypes.byref(self.prm), int(n_max), _stream_handle(self.device),
                                             ctypes.byref(self.ctx)))

    def close(self):
        if self.ctx:
            self.lib.hermite_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def state(self, mass, x, v, t=0.0):
        return DeviceState(self.p, mass, x, v, self.device, t)

    def restore(self, snap):
        """A state from ``DeviceState.host()`` output (checkpoint/resume), marked initialised."""
        st = DeviceState(self.p, snap["mass"], snap["x"], snap["v"], self.device, snap["t"])
        st.deriv.copy_(torch.as_tensor(np.stack(snap["derivs"])))
        if "cx" in snap:
            st.comp.copy_(torch.as_tensor(np.stack([snap["cx"], snap["cv"]])))
            st.c.t_comp = float(snap["t_comp"])
        st.mark_initialized()
        return st

    def use_current_stream(self):
        _check(self.ctx, self.lib.hermite_set_stream(self.ctx, _stream_handle(self.device)))

    def init(self, st):
        _check(self.ctx, self.lib.hermite_init(self.ctx, ctypes.byref(st.c)))

    def predict(self, st, dt):
        _check(self.ctx, self.lib.hermite_predict(self.ctx, ctypes.byref(st.c), float(dt)))

    def force_derivs(self, st):
        _check(self.ctx, self.lib.hermite_force_derivs(self.ctx, ctypes.byref(st.c)))

    def force_derivs_range(self, st, i0, ni):
        """The evaluation for i-particles [i0, i0 + ni) against all j (one GPU's
        share of an i-sharded evaluation); the rest of st.eval is left alone."""
        _check(self.ctx, self.lib.hermite_force_derivs_range(self.ctx, ctypes.byref(st.c), int(i0), int(ni)))

    def correct(self, st, dt, last_iter):
        _check(self.ctx, self.lib.hermite_correct(self.ctx, ctypes.byref(st.c), float(dt), 1 if last_iter else 0))

    def step(self, st, dt, n_iter):
        _check(self.ctx, self.lib.hermite_step(self.ctx, ctypes.byref(st.c), float(dt), int(n_iter)))

    def step_criterion(self, st, eta):
        """H = eta min over pairs of ((r^2 + eps^2)^(3/2) / (G (m_i + m_j)))^(1/2) at st.pos (Eq. 25)."""
        h = ctypes.c_double()
        _check(self.ctx, self.lib.hermite_step_criterion(self.ctx, ctypes.byref(st.c), float(eta), ctypes.byref(h)))
        return h.value

    def step_symmetric(self, st, eta, n_iter, direction=1.0):
        """One P(EC)^n step of implicit, time-symmetric length (H_- + H_+)/2 (Sec. 3.3); returns it."""
        dt = ctypes.c_double()
        _check(self.ctx, self.lib.hermite_step_symmetric(self.ctx, ctypes.byref(st.c), float(eta), int(n_iter),
                                                         float(direction), ctypes.byref(dt)))
        return dt.value

    def potential(self, st):
        phi = torch.empty(st.n, dtype=torch.float64, device=self.device)
        _check(self.ctx, self.lib.hermite_potential(self.ctx, ctypes.byref(st.c), ctypes.c_void_p(phi.data_ptr())))
        return phi

    def set_launch(self, i_per_thread, j_split, j_source=1, wg_waves=4):
        """j_source: 0 = LDS tiles, 1 = scalar stream (SGPR operands);
        wg_waves: 4 or 16 wave64 per workgroup."""
        _check(self.ctx, self.lib.hermite_set_launch(self.ctx, int(i_per_thread), int(j_split), int(j_source),
                                                     int(wg_waves)))

    def autotune(self, st):
        """Times the supported launch shapes; returns (i_per_thread, j_split, j_source, wg_waves)."""
        ipt, js, src, wv = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(self.ctx, self.lib.hermite_autotune(self.ctx, ctypes.byref(st.c), ctypes.byref(ipt), ctypes.byref(js),
                                                   ctypes.byref(src), ctypes.byref(wv)))
        return ipt.value, js.value, src.value, wv.value


class BatchHermite:
    """Batched form: many independent systems advanced in one persistent launch."""

    def __init__(self, order, offsets, precision="fp64", corrector="modified", G=1.0, eps2=0.0,
                 check_finite=False, device="cuda:0", compensated=False):
        self.lib = load_library()
        self.order = order
        self.p = order // 2 - 1
        self.device = torch.device(device)
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        self.n_sys = self.offsets.shape[0] - 1
        self.prm = Params(order, PRECISIONS[precision], CORRECTORS[corrector], 1 if check_finite else 0,
                          float(G), float(eps2), 1 if compensated else 0, 0)
        self.ctx = ctypes.c_void_p()
        _check(None, self.lib.hermite_batch_create(
            ctypes.byref(self.prm), int(self.n_sys),
            self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            _stream_handle(self.device), ctypes.byref(self.ctx)))

    def close(self):
        if self.ctx:
            self.lib.hermite_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def state(self, mass, x, v):
        return DeviceState(self.p, mass, x, v, self.device, with_pred=False)

    def init(self, st):
        _check(self.ctx, self.lib.hermite_batch_init(self.ctx, ctypes.byref(st.c)))

    def _dt_tensor(self, dt_sys):
        if not isinstance(dt_sys, torch.Tensor):
            dt_sys = torch.as_tensor(np.asarray(dt_sys, dtype=np.float64))
        dt_sys = dt_sys.to(device=self.device, dtype=torch.float64).contiguous()
        self._dt = dt_sys          # keep alive: the captured graph holds its address
        return dt_sys

    def set_launch(self, workgroups=0, waves=2, ring_min=57):
        """Batched launch shape (hermite_batch_set_launch): persistent workgroups
        (0: all resident), waves per bin (1, 2, 4), ring_min (whole-wave ring
        from this many bodies; 65: never)."""
        _check(self.ctx, self.lib.hermite_batch_set_launch(self.ctx, int(workgroups), int(waves), int(ring_min)))

    def get_launch(self):
        """The shape in use: (workgroups, waves, ring_min)."""
        v = [ctypes.c_int32() for _ in range(3)]
        _check(self.ctx, self.lib.hermite_batch_get_launch(self.ctx, *[ctypes.byref(q) for q in v]))
        return tuple(q.value for q in v)

    def autotune(self, st, dt_sys, n_steps, n_iter):
        """Times the supported shapes on a copy of st (hermite_batch_autotune);
        returns ((workgroups, waves, ring_min), from_cache)."""
        dt_sys = self._dt_tensor(dt_sys)
        v = [ctypes.c_int32() for _ in range(4)]
        _check(self.ctx, self.lib.hermite_batch_autotune(self.ctx, ctypes.byref(st.c),
                                                         ctypes.c_void_p(dt_sys.data_ptr()), int(n_steps),
                                                         int(n_iter), *[ctypes.byref(q) for q in v]))
        return tuple(q.value for q in v[:3]), bool(v[3].value)

    def run(self, st, dt_sys, n_steps, n_iter):
        """n_iter: one count for every system, or a sequence of one per system."""
        dt_sys = self._dt_tensor(dt_sys)
        if np.ndim(n_iter) == 0:
            _check(self.ctx, self.lib.hermite_batch_run(self.ctx, ctypes.byref(st.c),
                                                        ctypes.c_void_p(dt_sys.data_ptr()), int(n_steps),
                                                        int(n_iter)))
        else:
            it = np.ascontiguousarray(n_iter, dtype=np.int32)
            if it.shape != (self.n_sys,):
                raise ValueError("one n_iter per system")
            _check(self.ctx, self.lib.hermite_batch_run_iters(
                self.ctx, ctypes.byref(st.c), ctypes.c_void_p(dt_sys.data_ptr()), int(n_steps),
                it.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return dt_sys


class EnsembleHermite:
    """Ensemble form: independent systems of 2..128 bodies, each run by one
    workgroup with the variable time-symmetric step, many steps per launch."""

    def __init__(self, order, offsets, corrector="modified", G=1.0, eps2=0.0, device="cuda:0"):
        self.lib = load_library()
        self.order = order
        self.p = order // 2 - 1
        self.device = torch.device(device)
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        self.n_sys = self.offsets.shape[0] - 1
        self.prm = Params(order, 0, CORRECTORS[corrector], 0, float(G), float(eps2), 0, 0)
        self.ctx = ctypes.c_void_p()
        self.rec = None
        _check(None, self.lib.hermite_ensemble_create(
            ctypes.byref(self.prm), int(self.n_sys), self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            _stream_handle(self.device), ctypes.byref(self.ctx)))

    def close(self):
        if self.ctx:
            self.lib.hermite_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def state(self, mass, x, v):
        return DeviceState(self.p, mass, x, v, self.device, with_pred=False)

    def init(self, st, rec_cap=0):
        """Initial derivatives; system times and counters back to 0; a fresh
        (t, E) record buffer of rec_cap entries per system."""
        _check(self.ctx, self.lib.hermite_ensemble_init(self.ctx, ctypes.byref(st.c)))
        self.rec_cap = int(rec_cap)
        self.rec = torch.zeros((max(self.n_sys, 1), max(self.rec_cap, 1), 2), dtype=torch.float64,
                               device=self.device)

    def run(self, st, eta, t_end, n_iter, rec_from=float("inf"), max_steps=1 << 40):
        """Per-system (or scalar) eta, t_end, n_iter, rec_from.  Returns a list
        of dicts (t, E0, steps, records, failed, rec_overflow)."""
        cfg = (VstepCfg * max(self.n_sys, 1))()
        b = lambda q: np.broadcast_to(np.asarray(q), (self.n_sys,))
        for i, (e, te, ni, rf) in enumerate(zip(b(eta), b(t_end), b(n_iter), b(rec_from))):
            cfg[i] = VstepCfg(float(e), float(te), float(rf), int(ni), 0)
        res = (VstepResult * max(self.n_sys, 1))()
        _check(self.ctx, self.lib.hermite_ensemble_run(self.ctx, ctypes.byref(st.c), cfg, int(max_steps),
                                                       self.rec_cap, ctypes.c_void_p(self.rec.data_ptr()), res))
        return [dict(t=r.t, E0=r.E0, steps=r.steps, records=r.records, failed=r.failed,
                     rec_overflow=r.rec_overflow) for r in res[: self.n_sys]]

    def records(self, sys, count=None):
        """(t, E) records of one system as a numpy array [count][2]."""
        r = self.rec[sys].cpu().numpy()
        return r if count is None else r[:count]


def fma_rate(precision="fp64"):
    """Measured FMA issue rate of the current device (lane-FMA/s) in the
    accumulating form the evaluation's chains use: "fp64", or "fp32"
    (hermite_fma_rate)."""
    code = {"fp64": 0, "fp32": 1}[precision]   # HERMITE_FP64, HERMITE_MIXED
    r = ctypes.c_double(0.0)
    _check(None, load_library().hermite_fma_rate(code, ctypes.byref(r)))
    return r.value


def force_derivs_noalloc(order, st, precision="fp64", G=1.0, eps2=0.0, device="cuda:0"):
    """One evaluation along st.pred into st.eval without a context and without
    allocating (hermite_force_derivs_noalloc), on the current torch stream."""
    lib = load_library()
    prm = Params(int(order), PRECISIONS[precision], 0, 0, float(G), float(eps2), 0, 0)
    _check(None, lib.hermite_force_derivs_noalloc(ctypes.byref(prm), ctypes.byref(st.c),
                                                  _stream_handle(torch.device(device))))


def tune_cache_clear():
    """Forget the autotuners' cached picks of this process (hermite_tune_cache_clear)."""
    load_library().hermite_tune_cache_clear()


def version():
    return load_library().hermite_version().decode()
