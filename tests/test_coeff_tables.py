"""The GPU path's hard-coded corrector and interpolation constants
(paper_2006_02501_amd/csrc/hermite_coeffs.h) against the oracle's exact
solve of Eq. 8 and its numerical Hermite interpolation (CPU only)."""
import os
import re
from fractions import Fraction

import numpy as np
import pytest

from oracle import hermite_oracle as ho

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2006_02501_amd", "csrc", "hermite_coeffs.h")


def _array(name):
    src = open(HDR).read()
    m = re.search(r"\b%s\b[^=]*=\s*(\{.*?\});" % re.escape(name), src, flags=re.S)
    assert m, name
    body = re.sub(r"//[^\n]*", "", m.group(1))
    nums = re.findall(r"-?\d+\.\d+(?:\s*/\s*\d+\.\d+)?", body)

    def val(t):
        if "/" in t:
            a, b = t.split("/")
            return Fraction(a.strip()) / Fraction(b.strip())
        return Fraction(t.strip())
    return [val(t) for t in nums]


def test_velocity_table():
    cv = _array("CV")
    for p in (1, 2, 3):
        row = cv[4 * p: 4 * p + 4]
        assert row[: p + 1] == ho.endpoint_coefficients(p)
        assert all(c == 0 for c in row[p + 1:])


@pytest.mark.parametrize("ci,corr", [(0, "modified"), (1, "beta1"), (2, "shifted")])
def test_position_tables(ci, corr):
    cx = _array("CX")
    for p in (1, 2, 3):
        base = ci * 20 + p * 5
        row = cx[base: base + 5]
        assert row[: p + 2] == ho.endpoint_coefficients(p, ho.corrector_beta(p, corr))


def _interp_gpu_form(p, dt, a0, a1):
    if p == 2:
        A0, A1 = _array("I6_A0"), _array("I6_A1")
        num = sum((float(A0[m]) * a0[m] + float(A1[m]) * a1[m]) * dt ** m for m in range(3))
        return [num / dt ** 3]
    out = []
    for k, (n0, n1) in ((4, ("I8_4_A0", "I8_4_A1")), (5, ("I8_5_A0", "I8_5_A1"))):
        A0, A1 = _array(n0), _array(n1)
        num = sum((float(A0[m]) * a0[m] + float(A1[m]) * a1[m]) * dt ** m for m in range(4))
        out.append(num / dt ** k)
    return out


@pytest.mark.parametrize("p", [2, 3])
def test_interpolation_tables(p):
    rng = np.random.default_rng(p)
    dt = 0.37
    a0 = [rng.normal(size=5) for _ in range(p + 1)]
    a1 = [rng.normal(size=5) for _ in range(p + 1)]
    g = _interp_gpu_form(p, dt, a0, a1)
    o = ho.interpolate_higher(p, dt, a0, a1)
    for q, r in zip(g, o):
        assert np.allclose(q, r, rtol=1e-10, atol=1e-10 * np.abs(r).max())
