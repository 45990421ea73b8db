"""The FP64 exp2 polynomial in the kernel source (host only).

exp2_fp64 in csrc/vtx_kernels.hip evaluates 2^x as ldexp(P(f), n), f = x - n, with P the
degree-10 Chebyshev interpolant of 2^f on [-1/2, 1/2]. gen/exp2_coeffs.py derives P in 200-bit
arithmetic. Here: the constants in the source are the ones it derives, and the
evaluation in the kernel's order, with exact fma, is within 5e-16 of 200-bit 2^x, also at the
ends of the reduced interval and of the normal double range (subnormal results carry the
rounding of the subnormal format itself), and it gives +inf and 0 beyond the range (its callers
cap the argument at 1000, so +inf never reaches it).
"""
import math
import os
import re

import pytest

mpmath = pytest.importorskip("mpmath")

from paper_1404_1719_amd import build_lib  # noqa: E402
from paper_1404_1719_amd.gen import exp2_coeffs  # noqa: E402


def source_coefficients():
    src = open(os.path.join(build_lib.CSRC, "vtx_kernels.hip")).read()
    m = re.search(r"kExpPoly\[(\d+)\]\s*=\s*\{([^}]*)\}", src)
    assert m, "kExpPoly not found"
    vals = [float(v) for v in m.group(2).replace("\n", " ").split(",") if v.strip()]
    assert len(vals) == int(m.group(1))
    return vals


def test_source_constants_are_the_derived_ones():
    assert source_coefficients() == exp2_coeffs.coefficients()


def test_accuracy_of_the_evaluation():
    c = source_coefficients()
    assert exp2_coeffs.worst_error(c, samples=3000, seed=5) < 5e-16
    mpmath.mp.prec = 200
    for x in (-0.5, 0.5, -0.4999999999999999, 1e-300, -1022.0, -1021.3, 1023.75, 37.25):
        ref = mpmath.power(2, mpmath.mpf(x))
        assert abs((mpmath.mpf(exp2_coeffs.exp2(x, c)) - ref) / ref) < 5e-16, x


def test_limits():
    c = source_coefficients()
    assert exp2_coeffs.exp2(1024.0, c) == math.inf
    assert exp2_coeffs.exp2(5000.0, c) == math.inf and math.isfinite(exp2_coeffs.exp2(1000.0, c))
    assert exp2_coeffs.exp2(-1080.0, c) == 0.0 and exp2_coeffs.exp2(-math.inf, c) == 0.0
