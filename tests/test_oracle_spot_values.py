"""Pins of the oracle against literal values fixed outside it.

* Spot values (tests/golden/spot_values.txt): the angular weights H of scattering and pair
  annihilation at three electron energies, and the converged scattering and annihilation
  kernels at T = 10 MeV, eta_e = 5, each a number obtained by independent high-precision
  numeric integration of the definitions, asserted to its printed digits.
* The weak couplings against the textbook tree-level ones: for nu_e e scattering (charged and
  neutral current) g_L = 1/2 + s_W, g_R = s_W; for nu_mu e and nu_tau e g_L = -1/2 + s_W,
  g_R = s_W; an antineutrino swaps g_L and g_R. The cross-section of a massless target is
  sigma = (G_F^2 s / pi)(g_L^2 + g_R^2 / 3), so the non-degenerate total out-scattering rate of
  species s is e^eta (16 G_F^2 eps T^4 / pi^3)(g_L^2 + g_R^2 / 3), and nu_x (the mean of nu_mu
  and its antineutrino) has (2/3)(g_L^2 + g_R^2). The oracle's S-split rates are pinned to the
  S-split textbook rates elsewhere (e^eta 4 G_F^2 eps T^4 / pi^3 for S = I and a third of it for
  S = II); here its couplings combine them into the species rates, and its contraction
  combines the S-split kernels into the species opacities with the textbook couplings.
* sigma(nu_mu e) / E_nu for an electron at rest against its textbook size, 1.56e-42 cm^2/GeV.
"""
import math
import os

import numpy as np
import pytest
import scipy.integrate as si

from oracle import converged, physics, rates
from oracle.angular import h_nes, h_pair

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "spot_values.txt")
S_L = ((1, 0), (1, 1), (2, 0), (2, 1))


def spot_rows():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                p = line.split()
                rows.append((p[0], [float(v) for v in p[1:]]))
    return rows


def printed_tol(v, digits):
    """Half a unit in the last of the significant digits the values are printed to (H: 12,
    Phi: 10; trailing zeros dropped)."""
    return 0.5 * 10.0 ** (math.floor(math.log10(abs(v))) - (digits - 1))


def test_spot_values_of_the_angular_weights():
    n = 0
    for kind, v in spot_rows():
        if not kind.startswith("H_"):
            continue
        e, ep, E = v[:3]
        fn = h_nes if kind == "H_nes" else h_pair
        for (S, l), ref in zip(S_L, v[3:]):
            got = float(fn(l, S, e, ep, E))
            assert abs(got - ref) <= printed_tol(ref, 12) + 1e-12 * abs(ref), (kind, e, ep, E, S, l, got)
            n += 1
    assert n == 24


def test_spot_values_of_the_converged_kernels():
    n = 0
    g2 = physics.G_F ** 2
    for kind, v in spot_rows():
        if not kind.startswith("Phi_"):
            continue
        e, ep, T, eta = v[:4]
        for (S, l), ref in zip(S_L, v[4:]):
            if kind == "Phi_out":
                got = converged.nes_out(l, S, e, ep, T, eta * T) / g2
            else:
                got = converged.pair(l, S, e, ep, T, eta * T) / g2
            assert abs(got - ref) <= printed_tol(ref, 10) + 1e-11 * abs(ref), (kind, e, ep, S, l, got, ref)
            n += 1
    assert n == 12


def textbook_g(species, sin2w):
    """(g_L, g_R) of nu_e, anti-nu_e and nu_mu/nu_tau on electrons (tree level)."""
    ge = (0.5 + sin2w, sin2w)
    gm = (-0.5 + sin2w, sin2w)
    return {"nu_e": ge, "anti_nu_e": (ge[1], ge[0]), "nu_mu": gm, "anti_nu_mu": (gm[1], gm[0])}[species]


def textbook_factor(sin2w):
    """Species factors g_L^2 + g_R^2/3 of the non-degenerate rate, nu_x as the nu_mu mean."""
    def k(s):
        gl, gr = textbook_g(s, sin2w)
        return gl * gl + gr * gr / 3.0
    return (k("nu_e"), k("anti_nu_e"), 0.5 * (k("nu_mu") + k("anti_nu_mu")))


def oracle_species_factors(couplings):
    """beta_I + beta_II / 3 from the given couplings (the S-split rates are in ratio 1 : 1/3),
    over the 4 of beta = 4 g^2."""
    return tuple((b[0] + b[1] / 3.0) / 4.0 for b in couplings)


@pytest.mark.parametrize("sin2w", [0.2312, 0.25, 0.1])
def test_couplings_give_the_textbook_species_rates(sin2w):
    got = oracle_species_factors(physics.couplings(sin2w))
    ref = textbook_factor(sin2w)
    assert np.allclose(got, ref, rtol=1e-14, atol=0), (got, ref)
    # the measured-size ratio sigma(nu_e e) / sigma(nu_mu e) is about 6.1 at s_W = 0.2312
    if sin2w == 0.2312:
        gm = textbook_g("nu_mu", sin2w)
        assert 6.0 < ref[0] / (gm[0] ** 2 + gm[1] ** 2 / 3) < 6.3


def test_contraction_combines_species_with_the_textbook_couplings():
    """f = 0, scattering only: chi0 of species s is c0 sum_j w_j sum_S beta_S Phi_out_S(i, j);
    the betas must be the textbook 4 g_L^2, 4 g_R^2 (nu_x: 2 (g_L^2 + g_R^2) for both S)."""
    eps = np.array([3.0, 8.0, 20.0, 45.0])
    w = np.array([5.0, 40.0, 300.0, 2500.0])
    T, eta = np.array([4.0]), np.array([-2.0])
    opts = rates.Options(nquad=32, processes=rates.PROC_NES)
    f = np.zeros((1, 3, 2, 4))
    e, c = rates.forward(eps, w, T, eta, f, opts)
    k = rates.zone_kernels(eps, T, eta, opts)["nes_out"][0]   # [i, j, S, l]
    for s, name in enumerate(("nu_e", "anti_nu_e", None)):
        if name is None:
            gl, gr = textbook_g("nu_mu", physics.SIN2W)
            bI = bII = 2 * (gl * gl + gr * gr)
        else:
            gl, gr = textbook_g(name, physics.SIN2W)
            bI, bII = 4 * gl * gl, 4 * gr * gr
        ref = physics.C0 * np.sum(w[None, :] * (bI * k[:, :, 0, 0] + bII * k[:, :, 1, 0]), axis=1)
        assert np.allclose(c[0, s, 0], ref, rtol=1e-13, atol=0), (s, c[0, s, 0], ref)


def test_cross_section_size():
    """sigma(nu_mu e) / E_nu = 2 G_F^2 m_e (g_L^2 + g_R^2/3) / pi (hbar c)^2 ~ 1.56e-42 cm^2/GeV."""
    me = 0.51099895   # MeV
    gl, gr = textbook_g("nu_mu", physics.SIN2W)
    sig_per_mev = 2 * physics.G_F ** 2 * me * (gl * gl + gr * gr / 3) / math.pi * physics.HBARC ** 2
    assert abs(sig_per_mev * 1e3 / 1.56e-42 - 1) < 0.02
