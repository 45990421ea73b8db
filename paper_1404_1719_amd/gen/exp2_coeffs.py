"""Derive the polynomial of the FP64 exp2 in csrc/vtx_kernels.hip (exp2_fp64).

exp2_fp64 reduces 2^x to 2^n 2^f with n = rint(x) and f = x - n, |f| <= 1/2. This script
interpolates 2^f at the degree-10 Chebyshev nodes of [-1/2, 1/2] in 200-bit arithmetic,
converts the interpolant to monomial coefficients, rounds them to double, and checks the
resulting evaluation (Horner in f with exact fma emulated in rationals, then ldexp) against
200-bit 2^x.

Usage: python -m paper_1404_1719_amd.gen.exp2_coeffs   (prints the C initialiser)
Needs mpmath; it is not run by the build.
"""
import math
import random
from fractions import Fraction

import mpmath

DEGREE = 10


def coefficients(degree=DEGREE):
    mpmath.mp.prec = 200
    half = mpmath.mpf(1) / 2
    nodes = [half * mpmath.cos(mpmath.pi * (2 * k + 1) / (2 * (degree + 1))) for k in range(degree + 1)]
    vander = mpmath.matrix([[x ** j for j in range(degree + 1)] for x in nodes])
    values = mpmath.matrix([mpmath.power(2, x) for x in nodes])
    return [float(c) for c in mpmath.lu_solve(vander, values)]


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def exp2(x, c):
    """The kernel's evaluation order, with exact fma (the kernel's callers cap x at 1000)."""
    x = max(x, -2100.0)
    n = float(round(x))   # round half to even, as rint
    t = x - n
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
