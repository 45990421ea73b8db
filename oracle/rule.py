"""Quadrature rule R over the electron energy (oracle; test infrastructure only).

The workload descriptions fix only the node count ("32-point Gauss-Laguerre", "48-/64-point
quadrature"); the paper itself is silent on the rate quadrature. Reading used (identical on
the GPU side; its accuracy against adaptive integration is reported, not a parity target):

LAGUERRE (n-point, scattering only): E_k = T x_k, W_k = T w_k exp(x_k), with (x_k, w_k) the
  n-point Gauss-Laguerre rule; the pair kernel uses PANEL.
PANEL, scattering task (eps_i >= eps_j, Delta = eps_i - eps_j, mu = eta_e T):
  m = max(0, mu - Delta), u = max(0, mu), p = min(eps_j, u + KAPPA T),
  b_0 <= b_1 <= b_2 <= b_3 = sort(0, m, u, p);
  three Gauss-Legendre panels [b_0, b_1], [b_1, b_2], [b_2, b_3] and a Gauss-Laguerre tail
  E = b_3 + T x_k, n/4 nodes each. Zero-length panels keep their nodes (zero weight), so the
  rule is continuous in (T, eta_e).
PANEL, pair task (any i, j; w = eps_i + eps_j):
  sort(0, min(eps_i, eps_j), max(eps_i, eps_j), clip(mu, 0, w), w) -> four Gauss-Legendre
  panels of n/4 nodes. Tasks (i, j) and (j, i) get identical nodes.
Pins: tests/test_oracle_rule.py (exactness on monomials/exponentials, continuity, symmetry).
"""
import numpy as np
from numpy.polynomial import laguerre as _lag
from numpy.polynomial import legendre as _leg

KAPPA = 10.0
RULE_LAGUERRE = "laguerre"
RULE_PANEL = "panel"


def gauss_legendre01(m):
    """m-point Gauss-Legendre nodes/weights on [0, 1]."""
    x, w = _leg.leggauss(m)
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_laguerre_scaled(m):
    """m-point Gauss-Laguerre nodes x_k and weights w_k exp(x_k), for Integral_0^inf g(x) dx."""
    x, w = _lag.laggauss(m)
    return x, w * np.exp(x)


def _re(a):
    return np.real(a)


def _pos(a):
    """max(0, a), decided on the real part."""
    return np.where(_re(a) > 0, a, 0.0)


def _minimum(a, b):
    return np.where(_re(a) <= _re(b), a, b)


def _sort_last(stack):
    order = np.argsort(_re(stack), axis=-1, kind="stable")
    return np.take_along_axis(stack, order, axis=-1)


def _legendre_panels(bounds, m):
    """Nodes/weights of Gauss-Legendre panels between consecutive sorted breakpoints."""
    t, wt = gauss_legendre01(m)
    a = bounds[..., :-1, None]
    L = bounds[..., 1:, None] - a
    E = a + L * t
    W = L * wt
    return E.reshape(E.shape[:-2] + (-1,)), W.reshape(W.shape[:-2] + (-1,))


def nes_nodes(eps_i, eps_j, T, mu, n, rule=RULE_PANEL):
    """(E, W) of shape broadcast(eps_i, eps_j, T, mu) + (n,) for the scattering task eps_i >= eps_j."""
    eps_i, eps_j, T, mu = np.broadcast_arrays(np.asarray(eps_i, float), np.asarray(eps_j, float),
                                              np.asarray(T), np.asarray(mu))
    if rule == RULE_LAGUERRE:
        x, w = gauss_laguerre_scaled(n)
        return T[..., None] * x, T[..., None] * w
    if rule != RULE_PANEL or n % 4:
        raise ValueError("bad rule / node count")
    m4 = n // 4
    delta = eps_i - eps_j
    m = _pos(mu - delta)
    u = _pos(mu)
    p = _minimum(eps_j + 0 * u, u + KAPPA * T)
    zero = 0.0 * u
    b = _sort_last(np.stack(np.broadcast_arrays(zero, m, u, p), axis=-1))
    E1, W1 = _legendre_panels(b, m4)
    x, w = gauss_laguerre_scaled(m4)
    E2 = b[..., 3:4] + T[..., None] * x
    W2 = T[..., None] * w + 0 * E2
    return np.concatenate([E1, E2], axis=-1), np.concatenate([W1, W2], axis=-1)


def pair_nodes(eps_i, eps_j, T, mu, n):
    """(E, W) for the pair task (eps_i, eps_j); n/4 Gauss-Legendre nodes on each of 4 panels."""
    eps_i, eps_j, T, mu = np.broadcast_arrays(np.asarray(eps_i, float), np.asarray(eps_j, float),
                                              np.asarray(T), np.asarray(mu))
    if n % 4:
        raise ValueError("bad node count")
    w = eps_i + eps_j
    c = _minimum(_pos(mu), w + 0 * mu)
    zero = 0.0 * mu
    b = _sort_last(np.stack(np.broadcast_arrays(zero + 0 * w, np.minimum(eps_i, eps_j) + zero,
                                                np.maximum(eps_i, eps_j) + zero, c, w + zero), axis=-1))
    return _legendre_panels(b, n // 4)
