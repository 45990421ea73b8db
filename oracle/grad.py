"""Reverse-mode products of the rates (oracle; test infrastructure only).

The rates enter the Newton-Raphson solve of the implicit ray-by-ray transport step
(Sect. 2.1), which needs their derivatives with respect to the matter state and to f.

Given upstream gradients g_eta, g_chi [z, s, m, i], returns
  g_T[z]     = d/dT   sum(g_eta * eta + g_chi * chi)  at fixed eta_e,
  g_eta_e[z] = d/deta_e of the same at fixed T,
  g_f[z,s,m,j] = d/df of the same.
The derivatives are those of the discrete rule (node motion with T and mu_e = eta_e T
included), obtained by complex-step differentiation of ``oracle.rates``:
d/dx L = Im L(x + i h)/h, exact to rounding for h = 1e-30 |x|. The outputs are affine in f,
so the f-derivative uses the same step on each f entry with the kernels held fixed.
"""
import numpy as np

from .rates import Options, contract, zone_kernels

_H = 1e-30


def _objective(k, w, f, g_eta, g_chi, opts):
    e, c = contract(k, w, f, opts)
    return np.sum(g_eta * e + g_chi * c, axis=(1, 2, 3))


def vjp(eps, w, T, eta_e, f, g_eta, g_chi, opts=Options(), chunk=16):
    T = np.asarray(T, dtype=float)
    eta_e = np.asarray(eta_e, dtype=float)
    nz = T.shape[0]
    g_T = np.zeros(nz)
    g_e = np.zeros(nz)
    g_f = np.zeros_like(f)
    for z0 in range(0, nz, chunk):
        sl = slice(z0, z0 + chunk)
        Tz, ez, fz = T[sl], eta_e[sl], f[sl]
        ht = _H * Tz
        k = zone_kernels(eps, Tz + 1j * ht, ez, opts)
        g_T[sl] = np.imag(_objective(k, w, fz, g_eta[sl], g_chi[sl], opts)) / ht
        he = _H * np.maximum(np.abs(ez), 1.0)
        k = zone_kernels(eps, Tz, ez + 1j * he, opts)
        g_e[sl] = np.imag(_objective(k, w, fz, g_eta[sl], g_chi[sl], opts)) / he
        k = zone_kernels(eps, Tz, ez, opts)
        shape = fz.shape[1:]
        for d in range(int(np.prod(shape))):
            idx = np.unravel_index(d, shape)
            fc = fz.astype(complex)
            fc[(slice(None),) + idx] += 1j * _H
            g_f[(sl,) + idx] = np.imag(_objective(k, w, fc, g_eta[sl], g_chi[sl], opts)) / _H
    return g_T, g_e, g_f
