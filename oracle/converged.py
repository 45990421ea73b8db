"""Converged reference integrals (oracle; test infrastructure only).

Adaptive quadrature (scipy.integrate.quad, relative tolerance 1e-12) of the continuous
kernels, with breakpoints at every kink and transition of the integrand. It measures the
discretisation error of the rule R (reported, not a parity target) and checks the
continuous identities: Phi_out(e', e) = exp(-(e - e')/T) Phi_out(e, e') (time reversal)
and Phi_p = exp(-(e + e')/T) Phi_a (detailed balance), each integrated directly.
"""
import math

import numpy as np
import scipy.integrate as si

from . import physics
from .angular import h_nes, h_pair
from .rates import fermi, one_minus_fermi, one_minus_fermi_positron


def _quad(fun, pts, upper_inf):
    pts = sorted(set(float(p) for p in pts))
    tot = 0.0
    for a, b in zip(pts[:-1], pts[1:]):
        if b > a:
            tot += si.quad(fun, a, b, epsabs=0.0, epsrel=1e-12, limit=500)[0]
    if upper_inf:
        tot += si.quad(fun, pts[-1], np.inf, epsabs=0.0, epsrel=1e-12, limit=500)[0]
    return tot


def nes_out(l, S, e, ep, T, mu, production=False):
    """Continuous Phi_out_{l,S}(e -> ep) for any ordering of e, ep."""
    lo = max(0.0, ep - e)

    def g(E):
        return float(np.real(fermi(E, mu, T) * one_minus_fermi(E + e - ep, mu, T) * h_nes(l, S, e, ep, E)))

    pts = [lo, max(lo, ep), max(lo, mu), max(lo, mu - (e - ep)), max(lo, min(ep, mu) if mu > 0 else lo)]
    return physics.G_F ** 2 / (math.pi * e * ep) * _quad(g, pts, True)


def pair(l, S, e, ep, T, mu, production=False):
    """Continuous annihilation (or production) kernel Phi_{l,S}(e, ep)."""
    w = e + ep

    def g(E):
        if production:
            blk = fermi(E, mu, T) * (1.0 - one_minus_fermi_positron(w - E, mu, T))
        else:
            blk = one_minus_fermi(E, mu, T) * one_minus_fermi_positron(w - E, mu, T)
        return float(np.real(blk * h_pair(l, S, e, ep, E)))

    pts = [0.0, min(e, ep), max(e, ep), min(max(mu, 0.0), w), w]
    return physics.G_F ** 2 / (math.pi * e * ep) * _quad(g, pts, False)
