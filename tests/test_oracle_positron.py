"""Pins for neutrino-positron scattering in the oracle (process bit PROC_NPS).

* Non-degenerate positron gas: the total out-scattering rate of nu_e off positrons is
  e^{-eta_e} 4 G_F^2 eps T^4/pi^3 (beta_II + beta_I/3), the textbook cross-section
  sigma(nu e+) = (G_F^2 s/pi)(g_R^2 + g_L^2/3) averaged over a Maxwell-Boltzmann positron gas
  (the antiparticle target exchanges the roles of g_L and g_R against nu e-).
* CP conjugation: anti-nu_e on positrons at eta_e equals nu_e on electrons at -eta_e.
* The equilibrium null test covers the process (tests/test_oracle_rates.py).
"""
import math

import numpy as np

from oracle import physics, rates
from paper_1404_1719_amd import synth


def _row_rate(e, T, eta, b, nq=64):
    """(1/4pi^2) Integral eps'^2 Phi_out_0(e, eps') d eps' from the oracle's completed positron
    kernels on a grid of eps' quadrature nodes (split at the kink eps' = e)."""
    xg, wg = np.polynomial.legendre.leggauss(48)
    xl, wl = np.polynomial.laguerre.laggauss(32)
    ep1 = e * (xg + 1) / 2
    w1 = e / 2 * wg
    ep2 = e + T * xl
    w2 = T * wl * np.exp(xl)
    eps = np.concatenate([ep1, [e], ep2])
    wts = np.concatenate([w1, [0.0], w2])
    order = np.argsort(eps)
    eps, wts = eps[order], wts[order]
    ie = int(np.where(eps == e)[0][0])
    k = rates.zone_kernels(eps, np.array([T]), np.array([eta]), rates.Options(nquad=nq, processes=rates.PROC_NPS))
    _, pout = rates.scattering_kernels(k, b)
    return np.sum(wts * eps ** 2 * pout[0, ie, :, 0]) / (4 * math.pi ** 2)


def test_nondegenerate_positron_rate():
    e, T, eta = 11.0, 3.0, 40.0
    b = physics.couplings()[physics.NU_E]
    ref = math.exp(-eta) * 4 * physics.G_F ** 2 * e * T ** 4 / math.pi ** 3 * (b[1] + b[0] / 3)
    assert np.isclose(_row_rate(e, T, eta, b), ref, rtol=2e-6, atol=0)


def test_cp_conjugation():
    inp = synth.make_inputs("medium", nzones=3)
    b = physics.couplings()
    k_pos = rates.zone_kernels(inp.eps, inp.T, inp.eta_e, rates.Options(nquad=48, processes=rates.PROC_NPS))
    k_el = rates.zone_kernels(inp.eps, inp.T, -inp.eta_e, rates.Options(nquad=48, processes=rates.PROC_NES))
    for s, sc in ((physics.NU_EBAR, physics.NU_E), (physics.NU_E, physics.NU_EBAR), (physics.NU_X, physics.NU_X)):
        pin_p, pout_p = rates.scattering_kernels(k_pos, b[s])
        pin_e, pout_e = rates.scattering_kernels(k_el, b[sc])
        assert np.allclose(pout_p, pout_e, rtol=1e-14, atol=0)
        assert np.allclose(pin_p, pin_e, rtol=1e-14, atol=0)


def test_positrons_matter_only_where_they_exist():
    """At eta_e = 60 and T = 1 the positron rates are e^-60-suppressed against the electron ones;
    at eta_e = 0 they differ from them only by the coupling swap."""
    inp = synth.make_inputs("medium", nzones=2)
    inp.T[:] = [1.0, 5.0]
    inp.eta_e[:] = [60.0, 0.0]
    k = rates.zone_kernels(inp.eps, inp.T, inp.eta_e, rates.Options(nquad=48, processes=5))
    b = physics.couplings()[physics.NU_E]
    assert np.max(np.abs(k["nps_out"][0])) < 1e-20 * np.max(np.abs(k["nes_out"][0]))
    assert np.allclose(k["nps_out"][1], k["nes_out"][1], rtol=1e-14, atol=0)
    pin_both, _ = rates.scattering_kernels(k, b)
    assert np.allclose(pin_both[1], rates._species(k["nes_in"][1:], (b[0] + b[1], b[0] + b[1]))[0],
                       rtol=1e-12, atol=0)
