"""CPU checks of the C ABI: the library loads, exports every function that
include/hermite.h declares, and validates arguments before any HIP call
(no compute call is made here; no GPU is needed)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2006_02501_amd.hermite import Params, StateC, load_library

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hermite.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hermite_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_exported():
    lib = load_library()
    names = _declared()
    assert "hermite_force_derivs" in names and "hermite_step" in names
    for n in ("hermite_init", "hermite_predict", "hermite_correct", "hermite_batch_run"):
        assert n in names
    for n in names:
        assert hasattr(lib, n), n


def _create(**kw):
    lib = load_library()
    prm = dict(order=8, precision=0, corrector=0, check_finite=0, G=1.0, eps2=0.0, compensated=0)
    n_max = kw.pop("n_max", 16)
    prm.update(kw)
    p = Params(prm["order"], prm["precision"], prm["corrector"], prm["check_finite"], prm["G"], prm["eps2"],
               prm["compensated"], 0)
    ctx = ctypes.c_void_p()
    st = lib.hermite_create(ctypes.byref(p), n_max, None, ctypes.byref(ctx))
    return st, ctx


@pytest.mark.parametrize("kw,code", [
    (dict(order=5), -2), (dict(order=10), -2), (dict(order=0), -2),
    (dict(precision=3), -1), (dict(corrector=3), -1), (dict(corrector=-1), -1),
    (dict(eps2=-1e-9), -1), (dict(eps2=float("nan")), -1), (dict(G=float("inf")), -1),
    (dict(n_max=-1), -1), (dict(n_max=(1 << 40) + 1), -1), (dict(compensated=2), -1), (dict(compensated=-1), -1),
])
def test_create_rejects_bad_params(kw, code):
    st, ctx = _create(**kw)
    assert st == code
    assert not ctx.value


def test_create_null_out_and_null_params():
    lib = load_library()
    p = Params(8, 0, 0, 0, 1.0, 0.0)
    assert lib.hermite_create(ctypes.byref(p), 4, None, None) == -1
    ctx = ctypes.c_void_p()
    assert lib.hermite_create(None, 4, None, ctypes.byref(ctx)) == -1


def test_null_context_calls():
    lib = load_library()
    s = StateC()
    assert lib.hermite_init(None, ctypes.byref(s)) == -1
    assert lib.hermite_predict(None, ctypes.byref(s), 0.1) == -1
    assert lib.hermite_force_derivs(None, ctypes.byref(s)) == -1
    assert lib.hermite_force_derivs_range(None, ctypes.byref(s), 0, 1) == -1
    assert lib.hermite_correct(None, ctypes.byref(s), 0.1, 1) == -1
    assert lib.hermite_step(None, ctypes.byref(s), 0.1, 3) == -1
    assert lib.hermite_batch_run(None, ctypes.byref(s), None, 1, 1) == -1
    assert lib.hermite_set_launch(None, 1, 1, 0, 4) == -1
    assert lib.hermite_batch_set_launch(None, 0, 4, 57) == -1
    assert lib.hermite_batch_get_launch(None, None, None, None) == -1
    assert lib.hermite_batch_autotune(None, ctypes.byref(s), None, 1, 1, None, None, None, None) == -1
    lib.hermite_tune_cache_clear()
    assert lib.hermite_destroy(None) == 0
    assert lib.hermite_last_error(None)
    assert b"gfx950" in lib.hermite_version()


@pytest.mark.parametrize("offsets", [[0, 65], [0, 3, 3], [1, 4], [0, 5, 2]])
def test_batch_create_rejects_bad_layout(offsets):
    lib = load_library()
    p = Params(8, 0, 0, 0, 1.0, 0.0)
    off = np.array(offsets, dtype=np.int64)
    ctx = ctypes.c_void_p()
    st = lib.hermite_batch_create(ctypes.byref(p), len(offsets) - 1,
                                  off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), None, ctypes.byref(ctx))
    assert st == -1
    assert not ctx.value


@pytest.mark.parametrize("precision,compensated", [(2, 0), (2, 1)])
def test_batch_create_rejects_split(precision, compensated):
    lib = load_library()
    ctx = ctypes.c_void_p()
    p = Params(8, precision, 0, 0, 1.0, 0.0, compensated, 0)
    off = np.array([0, 3], dtype=np.int64)
    assert lib.hermite_batch_create(ctypes.byref(p), 1, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    None, ctypes.byref(ctx)) == -1
    assert not ctx.value


def test_struct_layouts_match_header(tmp_path):
    # the binding's ctypes structures against the C compiler's layout of the header
    fields = {Params: ("hermite_params", [f[0] for f in Params._fields_]),
              StateC: ("hermite_state", [f[0] for f in StateC._fields_])}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hermite.h"', "int main(void) {"]
    for cls, (cname, names) in fields.items():
        lines.append('printf("%%s %%zu\\n", "%s", sizeof(%s));' % (cname, cname))
        for f in names:
            lines.append('printf("%%s.%%s %%zu\\n", "%s", "%s", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                         check=True).stdout.splitlines())
    for cls, (cname, names) in fields.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f in names:
            assert int(got["%s.%s" % (cname, f)]) == getattr(cls, f).offset, (cname, f)


def test_batch_create_rejects_bad_order_and_null_offsets():
    lib = load_library()
    ctx = ctypes.c_void_p()
    p = Params(7, 0, 0, 0, 1.0, 0.0)
    off = np.array([0, 3], dtype=np.int64)
    assert lib.hermite_batch_create(ctypes.byref(p), 1, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    None, ctypes.byref(ctx)) == -2
    p = Params(8, 0, 0, 0, 1.0, 0.0)
    assert lib.hermite_batch_create(ctypes.byref(p), 1, None, None, ctypes.byref(ctx)) == -1


def test_fma_rate_rejects_bad_arguments():
    # argument checks come before any HIP call (no GPU needed)
    lib = load_library()
    r = ctypes.c_double(0.0)
    assert lib.hermite_fma_rate(2, ctypes.byref(r)) == -1
    assert lib.hermite_fma_rate(-1, ctypes.byref(r)) == -1
    assert lib.hermite_fma_rate(0, None) == -1
