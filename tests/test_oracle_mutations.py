"""Planted mistakes in the oracle (on the CPU, via monkeypatch) must trip its pins.

Each mutation is a plausible slip: a sign in the azimuthal average, a missing 1/2, the
positron chemical-potential sign, a dropped exp(x) in the Laguerre weights, an unswapped
anti-neutrino coupling. The matching pin is re-run against the mutated oracle."""
import math

import numpy as np
import pytest

import oracle.angular as ang
import oracle.physics as phys
import oracle.rates as rates
import oracle.rule as rule
from paper_1404_1719_amd import synth

import test_oracle_angular as pins_ang


def _brute_fails(l, S, e, ep, E, fn, avg, pole):
    ref = pins_ang.brute_h(avg, l, S, e, ep, E, pole)
    got = float(fn(l, S, e, ep, E))
    return abs(got - ref) > 5e-8 * abs(float(fn(0, S, e, ep, E)))


def test_sign_of_azimuthal_term(monkeypatch):
    orig = ang._phi_average
    monkeypatch.setattr(ang, "_phi_average", lambda *a: orig(*a[:-1], -a[-1]))
    assert _brute_fails(1, 1, 20.0, 10.0, 15.0, ang.h_nes, pins_ang.brute_nes_avg, 1.0)
    assert _brute_fails(0, 2, 20.0, 10.0, 25.0, ang.h_pair, pins_ang.brute_pair_avg, -1.0)


def test_missing_half_in_average(monkeypatch):
    def bad(e, ep, E, ca, cb, cbp, sbsb, sign):
        return ang.__dict__["_orig"](e, ep, E, ca, cb, cbp, sbsb * 2.0, sign)
    monkeypatch.setitem(ang.__dict__, "_orig", ang._phi_average)
    monkeypatch.setattr(ang, "_phi_average", bad)
    assert _brute_fails(0, 1, 20.0, 10.0, 5.0, ang.h_nes, pins_ang.brute_nes_avg, 1.0)


def test_positron_potential_sign(monkeypatch):
    monkeypatch.setattr(rates, "one_minus_fermi_positron", lambda E, mu, T: rates._sigma((E - mu) / T))
    inp = synth.make_inputs("medium", nzones=1)
    f = np.zeros((1, 3, 2, inp.eps.shape[0]))
    f[0, 0, 0] = 1 / (np.exp(inp.eps / inp.T[0] - 1.0) + 1)
    f[0, 1, 0] = 1 / (np.exp(inp.eps / inp.T[0] + 1.0) + 1)
    opts = rates.Options(nquad=48, processes=rates.PROC_PAIR)
    k = rates.zone_kernels(inp.eps, inp.T, inp.eta_e, opts)
    # detailed balance of the production kernel must break
    pf = np.exp(-(inp.eps[:, None] + inp.eps[None, :]) / inp.T[0])
    # the completed kernels still satisfy it by construction; a direct production quadrature does not
    E, W = rule.pair_nodes(inp.eps[3], inp.eps[5], inp.T[0], inp.eta_e[0] * inp.T[0], 48)
    mu, T, w = inp.eta_e[0] * inp.T[0], inp.T[0], inp.eps[3] + inp.eps[5]
    H = ang.h_pair(0, 1, inp.eps[3], inp.eps[5], E)
    ann = np.sum(W * rates.one_minus_fermi(E, mu, T) * rates.one_minus_fermi_positron(w - E, mu, T) * H)
    prod = np.sum(W * rates.fermi(E, mu, T) * (1 - rates.one_minus_fermi_positron(w - E, mu, T)) * H)
    assert not np.isclose(prod, pf[3, 5] * ann, rtol=1e-6, atol=0)


def test_laguerre_weights_without_exp(monkeypatch):
    orig = rule._lag.laggauss
    monkeypatch.setattr(rule, "gauss_laguerre_scaled", lambda m: orig(m))
    x, wt = rule.gauss_laguerre_scaled(12)
    assert not np.isclose(np.sum(wt * np.exp(-x) * x ** 3), math.factorial(3), rtol=1e-10, atol=0)


def test_unswapped_antineutrino_coupling(monkeypatch):
    good = phys.couplings()
    monkeypatch.setattr(phys, "couplings", lambda s=phys.SIN2W: (good[0], good[0], good[2]))
    b = phys.couplings()
    inp = synth.make_inputs("small", nzones=1)
    k = rates.zone_kernels(inp.eps, inp.T, inp.eta_e, rates.Options(nquad=32, rule="laguerre"))
    pa_nu = b[0][0] * k["pair_a"][..., 0, :] + b[0][1] * k["pair_a"][..., 1, :]
    pa_bar = b[1][0] * k["pair_a"][..., 0, :] + b[1][1] * k["pair_a"][..., 1, :]
    assert not np.allclose(pa_bar, np.swapaxes(pa_nu, 1, 2), rtol=1e-6, atol=0)


def test_transposed_pair_jacobian_block(monkeypatch):
    import test_oracle_jacobian as pins_jac
    orig = rates.jacobian_blocks

    def bad(kernels, w, opts, absolute=False):
        j = orig(kernels, w, opts, absolute)
        j[:, :, 1] = np.swapaxes(j[:, :, 1], -1, -2)
        return j
    monkeypatch.setattr(rates, "jacobian_blocks", bad)
    with pytest.raises(AssertionError):
        pins_jac.test_jacobian_reproduces_contraction("medium", 48, rule.RULE_PANEL)


def test_production_sign_in_jacobian(monkeypatch):
    import test_oracle_jacobian as pins_jac
    orig = rates.jacobian_blocks

    def bad(kernels, w, opts, absolute=False):
        j = orig(kernels, w, opts, absolute)
        j[:, :, 1, 2] *= -1.0
        return j
    monkeypatch.setattr(rates, "jacobian_blocks", bad)
    with pytest.raises(AssertionError):
        pins_jac.test_jacobian_transpose_is_f_gradient()


def test_unswapped_positron_couplings(monkeypatch):
    import test_oracle_positron as pins_pos

    def bad(kernels, b):
        pin = pout = 0.0
        for name in ("nes", "nps"):
            if name + "_out" in kernels:
                pin = pin + rates._species(kernels[name + "_in"], b)
                pout = pout + rates._species(kernels[name + "_out"], b)
        return pin, pout
    monkeypatch.setattr(rates, "scattering_kernels", bad)
    with pytest.raises(AssertionError):
        pins_pos.test_nondegenerate_positron_rate()


def test_positron_scattering_with_electron_potential(monkeypatch):
    import test_oracle_positron as pins_pos
    orig = rates.scattering_quadrature
    calls = []

    def bad(eps, T, mu, opts, absolute=False):
        calls.append(1)
        return orig(eps, T, np.abs(mu), opts, absolute)     # positron tasks at +mu_e
    monkeypatch.setattr(rates, "scattering_quadrature", bad)
    with pytest.raises(AssertionError):
        pins_pos.test_nondegenerate_positron_rate()


def test_interpolation_with_swapped_fractions(monkeypatch):
    import oracle.tabulated as tab
    import test_oracle_tabulated as pins_tab
    orig = tab.bilinear

    def bad(table, lat, T, eta_e):
        flip = tab.Lattice(lat.nt, lat.nh, lat.lnT0, lat.dlnT * 1.0000001, lat.eta0, lat.deta)
        return orig(table, flip, T, eta_e)
    monkeypatch.setattr(tab, "bilinear", bad)
    with pytest.raises(AssertionError):
        pins_tab.test_exact_on_bilinear_data()


def _cv_flipped_couplings(sin2w=phys.SIN2W, electron_mass=False):
    """nu_e with the nu_mu vector coupling C_V = -1/2 + 2 s_W (a dropped charged-current term)."""
    cv = -0.5 + 2.0 * sin2w
    b_e = ((cv + 0.5) ** 2, (cv - 0.5) ** 2)
    good = _GOOD_COUPLINGS(sin2w)
    return (b_e, (b_e[1], b_e[0]), good[2])


_GOOD_COUPLINGS = phys.couplings


def _unaveraged_nux(sin2w=phys.SIN2W, electron_mass=False):
    """nu_x as nu_mu alone (no average over particle and antiparticle)."""
    good = _GOOD_COUPLINGS(sin2w)
    cv = -0.5 + 2.0 * sin2w
    return (good[0], good[1], ((cv - 0.5) ** 2, (cv + 0.5) ** 2))


@pytest.mark.parametrize("bad", [_cv_flipped_couplings, _unaveraged_nux])
def test_wrong_couplings_trip_the_textbook_pins(monkeypatch, bad):
    import test_oracle_spot_values as pins_spot
    monkeypatch.setattr(phys, "couplings", bad)
    with pytest.raises(AssertionError):
        pins_spot.test_couplings_give_the_textbook_species_rates(0.2312)
    with pytest.raises(AssertionError):
        pins_spot.test_contraction_combines_species_with_the_textbook_couplings()


def test_wrong_azimuthal_half_trips_the_spot_values(monkeypatch):
    import test_oracle_spot_values as pins_spot

    def bad(e, ep, E, ca, cb, cbp, sbsb, sign):
        return ang.__dict__["_orig"](e, ep, E, ca, cb, cbp, sbsb * 2.0, sign)
    monkeypatch.setitem(ang.__dict__, "_orig", ang._phi_average)
    monkeypatch.setattr(ang, "_phi_average", bad)
    with pytest.raises(AssertionError):
        pins_spot.test_spot_values_of_the_angular_weights()


def test_short_interval_route_slips(monkeypatch):
    """The direct-integrand route of short momentum-transfer intervals: too few Gauss points,
    or 1 - x without its factor 1/2, must fail the brute-force pins of the short cases."""
    e, ep, E = pins_ang.CASES_NES_SHORT[1]
    x2, w2 = np.polynomial.legendre.leggauss(2)
    monkeypatch.setattr(ang, "_GL_X", x2)
    monkeypatch.setattr(ang, "_GL_W", w2)
    assert _brute_fails(1, 1, e, ep, E, ang.h_nes, pins_ang.brute_nes_avg, 1.0)
    e, ep, E = pins_ang.CASES_PAIR_SHORT[0]
    assert _brute_fails(1, 2, e, ep, E, ang.h_pair, pins_ang.brute_pair_avg, -1.0)
    monkeypatch.undo()
    orig = ang._nes_direct

    def bad(l, S, e, ep, E, k):
        # the Legendre factor of l = 1 with 1 - x = Q^2/(e e') instead of Q^2/(2 e e')
        val0 = orig(0, S, e, ep, E, k)
        if l == 0:
            return val0
        om = e - ep
        x_bad = 1 - (k * k - om * om) / (e * ep)
        return x_bad * val0
    monkeypatch.setattr(ang, "_nes_direct", bad)
    e, ep, E = pins_ang.CASES_NES_SHORT[0]
    assert _brute_fails(1, 1, e, ep, E, ang.h_nes, pins_ang.brute_nes_avg, 1.0)


def test_newton_source_jacobian_slips(monkeypatch):
    """The source's derivative without the factor 3 of the f1 coupling, or with the blocks of the
    pair's partner species taken from the species itself, must fail the finite-difference pin."""
    import oracle.newton as onewton
    import test_oracle_newton as pins_newton
    orig = onewton.source_jacobian

    def no_three(jac, f, eta, chi):
        dS = orig(jac, f, eta, chi)
        nz, B = dS.shape[0], dS.shape[1]
        ne = B // 6
        d = dS.reshape(nz, 3, 2, ne, 3, 2, ne)
        for s in range(3):
            for i in range(ne):
                d[:, s, 0, i, s, 1, i] += 2.0 / 3.0 * 3.0 * chi[:, s, 1, i]   # -3 chi1 -> -chi1
        return d.reshape(nz, B, B)
    monkeypatch.setattr(onewton, "source_jacobian", no_three)
    with pytest.raises(AssertionError):
        pins_newton.test_diagonal_blocks_are_the_residual_derivative()
    monkeypatch.setattr(onewton, "SOURCE", ((0, 1, 2), (0, 1, 2)))
    monkeypatch.setattr(onewton, "source_jacobian", orig)
    with pytest.raises(AssertionError):
        pins_newton.test_source_jacobian_from_the_rates_blocks()


def test_massive_weight_slips(monkeypatch):
    """Electron-mass weights: massless kinematics in the azimuthal angle (P -> E), the positron's
    momentum taken equal to the electron's, and a doubled mass structure must each trip the
    four-vector brute force or the vacuum pair cross-section."""
    import oracle.massive as mas
    import test_oracle_massive as pins_mas

    def fails_nes(l, S, e, ep, E):
        ref = pins_mas.brute_h(pins_mas.brute_nes_avg, l, S, e, ep, E, 1.0)
        return abs(float(mas.h_nes(l, S, e, ep, E)) - ref) > 5e-8 * abs(float(mas.h_nes(0, 1, e, ep, E)))

    def fails_pair(l, S, e, ep, E):
        ref = pins_mas.brute_h(pins_mas.brute_pair_avg, l, S, e, ep, E, -1.0)
        return abs(float(mas.h_pair(l, S, e, ep, E)) - ref) > 5e-8 * abs(float(mas.h_pair(0, 1, e, ep, E)))

    nes, pair = mas._nes_integrand, mas._pair_integrand
    with monkeypatch.context() as mp:
        mp.setattr(mas, "_nes_integrand", lambda l, S, e, ep, E, P, m, k: nes(l, S, e, ep, E, E, m, k))
        assert fails_nes(0, 1, 2.0, 1.0, 0.8)
    with monkeypatch.context() as mp:
        mp.setattr(mas, "_pair_integrand", lambda l, S, e, ep, E, P, Pb, m, k: pair(l, S, e, ep, E, P, P, m, k))
        assert fails_pair(1, 2, 2.0, 1.0, 0.8)
    with monkeypatch.context() as mp:
        mp.setattr(mas, "_pair_integrand",
                   lambda l, S, e, ep, E, P, Pb, m, k: pair(l, S, e, ep, E, P, Pb, m, k) * (2.0 if S == 3 else 1.0))
        f = lambda E: float(mas.h_pair(0, 3, 1.0, 0.3, E))
        got = si_quad(f, mas.ME, 1.3 - mas.ME)
        assert abs(got - pins_mas._vacuum_closed(1.0, 0.3, 3, 0)) > 1e-6 * abs(got)


def si_quad(f, a, b):
    import scipy.integrate as si
    pts = np.linspace(a, b, 9)
    return sum(si.quad(f, x, y, epsabs=0, epsrel=1e-12, limit=400)[0] for x, y in zip(pts[:-1], pts[1:]))
