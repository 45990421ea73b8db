"""Pins for the oracle's rates with the electron mass (oracle.massive rule and quadratures,
completed and contracted by oracle.rates with the third structure).

* vacuum pair annihilation through the massive rule (T -> 0, mu = 0, so every blocking
  factor is 1): the task values equal G_F^2/(pi eps eps') times the phase-space tensor closed
  form of the pin on the weights, structure I and the symmetric third structure with its plus
  sign, at and below the pair threshold;
* cold dilute electron gas (T = 1e-6 MeV, mu_e = m - 10 T): electrons at rest, so the
  species-summed l = 0 scattering kernel is proportional to the textbook elastic cross-section
  beta_I eps^2 + beta_II eps'^2 - beta_III m (eps - eps'); its ratio between nu_e and nu_x is
  free of the common factor and fixes the sign of the mass term in the rates and the species
  sums;
* equilibrium null test and discrete detailed balance with the mass (the completion steps are
  exact for any rule and weights);
* the rule against a composite Gauss reference of the same integrand (a reported
  discretisation error, loose bound).
"""
import math

import numpy as np
import pytest
import scipy.integrate as si

from oracle import massive, physics, rates
from paper_1404_1719_amd import synth

import test_oracle_massive as pins

M = massive.ME


def test_couplings_with_mass():
    b = physics.couplings(physics.SIN2W, True)
    cv = 0.5 + 2 * physics.SIN2W
    cvx = -0.5 + 2 * physics.SIN2W
    assert b[0][2] == b[1][2] and np.isclose(b[0][2], (cv - 0.5) * (cv + 0.5), rtol=1e-15)
    assert np.isclose(b[2][2], (cvx - 0.5) * (cvx + 0.5), rtol=1e-15) and b[2][2] < 0
    assert [x[:2] for x in b] == list(physics.couplings(physics.SIN2W))


def test_vacuum_pair_through_the_rule():
    eps = np.array([0.3, 0.5, 0.6, 1.0, 10.0, 20.0])   # 0.3 x 0.5 < m^2: below threshold
    opts = rates.Options(nquad=128, electron_mass=True, processes=rates.PROC_PAIR)
    A, A3 = massive.pair_quadrature(eps, np.array([1e-6]), np.array([0.0]), opts)
    for i, e in enumerate(eps):
        for j, ep in enumerate(eps):
            for l in (0, 1):
                for S, arr in ((1, A), (3, A3)):
                    ref = physics.G_F ** 2 / (math.pi * e * ep) * pins._vacuum_closed(e, ep, S, l)
                    got = arr[0, i, j, l]
                    if ref == 0.0:
                        assert got == 0.0, (e, ep, S, l, got)
                    else:
                        assert abs(got - ref) <= 1e-10 * abs(ref), (e, ep, S, l, got, ref)


@pytest.mark.parametrize("i,j", [(3, 0), (2, 1), (3, 2), (1, 0)])
def test_cold_gas_species_ratio(i, j):
    eps = np.array([2.0, 3.0, 5.0, 8.0])
    T = 1e-6
    opts = rates.Options(nquad=48, electron_mass=True, processes=rates.PROC_NES)
    k = rates.zone_kernels(eps, np.array([T]), np.array([(M - 10 * T) / T]), opts)
    b = physics.couplings(physics.SIN2W, True)
    e, ep = eps[i], eps[j]
    phi = [rates._species(k["nes_out"], b[s])[0, i, j, 0] for s in (0, 2)]
    pred = [b[s][0] * e * e + b[s][1] * ep * ep - b[s][2] * M * (e - ep) for s in (0, 2)]
    assert phi[1] > 0
    assert abs((phi[0] / phi[1]) / (pred[0] / pred[1]) - 1) <= 2e-6


def _equilibrium_f(eps, T, amu):
    return 1.0 / (np.exp(eps / T - amu) + 1.0)


def test_equilibrium_null_with_mass():
    inp = synth.make_inputs("medium", nzones=3)
    eps, w = inp.eps, inp.w
    T = np.array([0.8, 2.0, 5.0])
    eta = np.array([1.0, 4.0, 12.0])
    for proc in (rates.PROC_NES, rates.PROC_PAIR, rates.PROC_NPS, 7):
        opts = rates.Options(nquad=48, processes=proc, electron_mass=True)
        f = np.zeros((3, 3, 2, eps.shape[0]))
        for z in range(3):
            a = 1.5 * z - 1.0
            f[z, 0, 0] = _equilibrium_f(eps, T[z], a)
            f[z, 1, 0] = _equilibrium_f(eps, T[z], -a)
            f[z, 2, 0] = _equilibrium_f(eps, T[z], 0.0)
        e, c, ae, ac = rates.forward_with_scale(eps, w, T, eta, f, opts)
        S0 = e[:, :, 0] - c[:, :, 0] * f[:, :, 0]
        assert np.all(ae[:, :, 0] > 0)
        assert np.all(np.abs(S0) <= 1e-13 * (ae[:, :, 0] + ac[:, :, 0]))


def test_discrete_detailed_balance_with_mass():
    inp = synth.make_inputs("medium", nzones=2)
    opts = rates.Options(nquad=48, electron_mass=True, processes=7)
    k = rates.zone_kernels(inp.eps, inp.T, inp.eta_e, opts)
    ne = inp.eps.shape[0]
    assert k["nes_out"].shape[-2] == 3 and k["pair_a"].shape[-2] == 3
    for z in range(2):
        for i in range(ne):
            for j in range(ne):
                fac = math.exp((inp.eps[j] - inp.eps[i]) / inp.T[z])
                if fac < 1e200:
                    assert np.allclose(k["nes_in"][z, i, j], fac * k["nes_out"][z, i, j], rtol=1e-12, atol=1e-300)
                pf = math.exp(-(inp.eps[i] + inp.eps[j]) / inp.T[z])
                assert np.allclose(k["pair_p"][z, i, j], pf * k["pair_a"][z, i, j], rtol=1e-12, atol=0)
                # the third structure of the pair is symmetric, the first two transpose
                assert np.isclose(k["pair_a"][z, i, j, 2, 0], k["pair_a"][z, j, i, 2, 0], rtol=1e-13, atol=0)
                assert k["pair_a"][z, i, j, 1, 1] == k["pair_a"][z, j, i, 0, 1]


def _converged_nes(l, S, e, ep, T, mu):
    """Composite Gauss-Legendre reference, independent of the rule's node layout: 16 panels of
    24 nodes on each segment between the integrand's breakpoints (E = m + L s^2 on the segment
    at the threshold), and on [b, b + 60 T] above the last one (the rest is below e^-50)."""
    om = e - ep
    ek = float(massive.nes_kink(e, ep))
    pts = sorted({M, ek, max(M, mu), max(M, mu - om)})
    x, wx = np.polynomial.legendre.leggauss(24)
    t = np.concatenate([(k + 0.5 * (x + 1)) / 16 for k in range(16)])
    wt = np.concatenate([0.5 * wx / 16] * 16)
    Es, Ws = [], []
    for a, b in zip(pts[:-1] + [pts[-1]], pts[1:] + [pts[-1] + 60 * T]):
        if a == M:
            Es.append(a + (b - a) * t * t)
            Ws.append(2 * (b - a) * t * wt)
        else:
            Es.append(a + (b - a) * t)
            Ws.append((b - a) * wt)
    E, W = np.concatenate(Es), np.concatenate(Ws)
    B = rates.fermi(E, mu, T) * rates.one_minus_fermi(E + om, mu, T)
    return physics.G_F ** 2 / (math.pi * e * ep) * np.sum(W * B * massive.h_nes(l, S, e, ep, E))


def test_rule_against_converged_with_mass():
    """Rule against a composite Gauss reference: a reported discretisation error (measured at
    most 2.7e-6 at 48 nodes, 1.1e-7 at 64), loose bound."""
    eps = np.array([2.5, 6.0, 25.0])
    errs = []
    for T, eta in [(1.0, 2.0), (0.6, 8.0), (3.0, 1.0)]:
        opts = rates.Options(nquad=48, electron_mass=True, processes=rates.PROC_NES)
        q = massive.scattering_quadrature(eps, np.array([T]), np.array([eta * T]), opts)
        ii, jj = rates.nes_tasks(3)
        for t, (i, j) in enumerate(zip(ii, jj)):
            for l in (0, 1):
                ref = _converged_nes(l, 1, eps[i], eps[j], T, eta * T)
                errs.append(abs(q[0, t, 0, l] - ref) / abs(ref))
    assert max(errs) < 1e-5, max(errs)
