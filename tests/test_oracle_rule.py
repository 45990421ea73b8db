"""Pins for the quadrature rule R (oracle.rule): exactness of the Gauss rules, panel layout,
continuity in (T, eta_e) and the pair-task symmetry."""
import math

import numpy as np
import pytest

from oracle import rule


@pytest.mark.parametrize("m", [8, 12, 16])
def test_gauss_legendre_exact(m):
    t, w = rule.gauss_legendre01(m)
    for p in range(2 * m):
        assert np.isclose(np.sum(w * t ** p), 1.0 / (p + 1), rtol=1e-13, atol=0)


@pytest.mark.parametrize("m", [8, 12, 16, 32])
def test_gauss_laguerre_exact(m):
    x, wt = rule.gauss_laguerre_scaled(m)
    for p in range(2 * m):
        # Integral_0^inf x^p e^-x dx = p!  (weights carry exp(x_k): integrand is x^p e^-x)
        assert np.isclose(np.sum(wt * np.exp(-x) * x ** p), math.factorial(p), rtol=1e-10, atol=0)


def test_nes_panel_layout():
    # eps_i = 30, eps_j = 20, T = 2, mu = 26: m = 16, u = 26, p = min(20, 46) = 20
    E, W = rule.nes_nodes(30.0, 20.0, 2.0, 26.0, 48)
    assert E.shape == (48,)
    b = [0.0, 16.0, 20.0, 26.0]
    t, wt = rule.gauss_legendre01(12)
    for g in range(3):
        np.testing.assert_allclose(E[12 * g:12 * g + 12], b[g] + (b[g + 1] - b[g]) * t, rtol=1e-14)
        np.testing.assert_allclose(W[12 * g:12 * g + 12], (b[g + 1] - b[g]) * wt, rtol=1e-14)
    x, wx = rule.gauss_laguerre_scaled(12)
    np.testing.assert_allclose(E[36:], 26.0 + 2.0 * x, rtol=1e-14)
    np.testing.assert_allclose(W[36:], 2.0 * wx, rtol=1e-14)
    # eps_j far above mu: decay panel capped at u + KAPPA T, kink left inside the tail
    E, W = rule.nes_nodes(300.0, 250.0, 1.0, 5.0, 48)
    assert np.isclose(E[36] - E[24:36].max(), 1.0 * x[0] + (15.0 - E[24:36].max()), rtol=1e-12, atol=0)


def test_rule_integrates_exp_poly():
    """Whole scattering rule on g(E) = E^2 exp(-E/T): Legendre panels are accurate, tail exact."""
    T, mu = 3.0, 20.0
    E, W = rule.nes_nodes(50.0, 8.0, T, mu, 64)
    g = E ** 2 * np.exp(-E / T)
    assert np.isclose(np.sum(W * g), 2 * T ** 3, rtol=1e-10, atol=0)


def test_continuity_in_mu():
    """Breakpoints reorder as mu sweeps through eps_j and eps_j + Delta; the rule stays continuous."""
    def val(mu):
        E, W = rule.nes_nodes(40.0, 25.0, 4.0, mu, 48)
        return np.sum(W * E ** 3 / (1 + np.exp((E - mu) / 4.0)))
    for mu0 in (25.0, 40.0, 65.0):   # mu = eps_j, mu - Delta = eps_j, mu = eps_j + ... crossings
        a, b = val(mu0 - 1e-9), val(mu0 + 1e-9)
        assert abs(a - b) <= 1e-7 * abs(a)


def test_pair_nodes_symmetric():
    for (a, b, mu) in [(3.0, 40.0, 10.0), (40.0, 3.0, 10.0), (12.0, 12.0, 50.0), (8.0, 30.0, -5.0)]:
        E1, W1 = rule.pair_nodes(a, b, 2.0, mu, 32)
        E2, W2 = rule.pair_nodes(b, a, 2.0, mu, 32)
        np.testing.assert_array_equal(E1, E2)
        np.testing.assert_array_equal(W1, W2)
        assert np.isclose(W1.sum(), a + b, rtol=1e-14, atol=0)
