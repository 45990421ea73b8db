"""Derive the polynomial of the FP64 exp2 in csrc/vtx_kernels.hip (exp2_fp64).

exp2_fp64 reduces 2^x to 2^n e^t with n = rint(x) and t = (x - n) ln 2, |t| <= ln2/2. This
script interpolates e^t at the degree-10 Chebyshev nodes of [-ln2/2, ln2/2] in 200-bit
arithmetic, converts the interpolant to monomial coefficients, rounds them to double, and
checks the resulting evaluation (Horner with exact fma emulated in rationals, then ldexp)
against 200-bit 2^x: the worst relative error is 4.2e-16.

Usage: python -m paper_1404_1719_amd.gen.exp2_coeffs   (prints the C initialiser)
Needs mpmath; it is not run by the build.
"""
import math
import random
from fractions import Fraction

import mpmath

DEGREE = 10
LN2 = 0.6931471805599453


def coefficients(degree=DEGREE):
    mpmath.mp.prec = 200
    half = mpmath.log(2) / 2
    nodes = [half * mpmath.cos(mpmath.pi * (2 * k + 1) / (2 * (degree + 1))) for k in range(degree + 1)]
    vander = mpmath.matrix([[x ** j for j in range(degree + 1)] for x in nodes])
    values = mpmath.matrix([mpmath.exp(x) for x in nodes])
    return [float(c) for c in mpmath.lu_solve(vander, values)]


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def exp2(x, c):
    """The kernel's evaluation order, with exact fma (the kernel's callers cap x at 1000)."""
    x = max(x, -2100.0)
    n = float(round(x))   # round half to even, as rint
    t = (x - n) * LN2
    p = c[-1]
    for k in range(len(c) - 2, -1, -1):
        p = _fma(p, t, c[k])
    try:
        return math.ldexp(p, int(n))
    except OverflowError:
        return math.inf


def worst_error(c, samples=20000, seed=2):
    mpmath.mp.prec = 200
    rng = random.Random(seed)
    xs = [rng.uniform(-1020, 1020) for _ in range(samples)] + [k / 64.0 for k in range(-64, 65)]
    worst = 0.0
    for x in xs:
        ref = mpmath.power(2, mpmath.mpf(x))
        worst = max(worst, float(abs((mpmath.mpf(exp2(x, c)) - ref) / ref)))
    return worst


if __name__ == "__main__":
    c = coefficients()
    print("constexpr double kExpPoly[%d] = {%s};" % (len(c), ", ".join(repr(v) for v in c)))
    print("// worst relative error of exp2: %.2e" % worst_error(c))
