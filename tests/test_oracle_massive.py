"""Pins for the oracle's angular weights with the electron mass (oracle.massive).

* massless limit: at m -> 0 the weights are the massless ones (oracle.angular, itself pinned by
  brute force and closed forms), and the third structure vanishes;
* brute force: explicit massive four-vectors (E^2 - P^2 = m^2 checked on both electrons), the
  azimuthal average on a uniform phi grid and adaptive quadrature in x = cos(q, q') over the
  region found numerically, for all three structures, l = 0 and 1, near and far from the
  thresholds;
* vacuum pair cross-section with the mass: the two-body phase-space tensor
  Integral dPhi p^mu pbar^nu = Phi [s beta^2/12 g^{mu nu} + (3 - beta^2)/12 Q^mu Q^nu],
  Phi = pi beta / 2, beta = sqrt(1 - 4 m^2 / s), contracted with the neutrino momenta, gives
  Integral dE H^{P,S}_l = Integral dx P_l(x) beta s^2 (3 + beta^2)/48  (S = I, II) and
  Integral dx P_l(x) beta m^2 s / 2  (S = III), s = 2 eps eps' (1 - x), zero below s = 4 m^2:
  this fixes the threshold and the beta dependence independently of the oracle's angles;
* electron at rest (E -> m): the weights reduce to the textbook elastic cross-section
  d sigma/dT ~ g_L^2 + g_R^2 (1 - T/eps)^2 - g_L g_R m T/eps^2 (T = eps - eps'), so
  H^II/H^I -> (eps'/eps)^2 and H^III/H^I -> m (eps - eps')/eps^2;
* time reversal and pair transposition, as for the massless weights.
"""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.optimize as so

from oracle import angular, massive

M = massive.ME


def mdot(a, b):
    return a[0] * b[0] - np.dot(a[1:], b[1:])


def frame(axis):
    k = axis / np.linalg.norm(axis)
    t = np.array([1.0, 0.0, 0.0]) if abs(k[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(k, t)
    e1 /= np.linalg.norm(e1)
    return k, e1, np.cross(k, e1)


NPHI = 16


def _neutrinos(e, ep, x):
    q3 = e * np.array([0.0, 0.0, 1.0])
    qp3 = ep * np.array([np.sqrt(1 - x * x), 0.0, x])
    return q3, qp3, np.concatenate([[e], q3]), np.concatenate([[ep], qp3])


def _structure(S, a, b, q, qp, m):
    """(q.a)(q'.b) for S = I, (q.b)(q'.a) for S = II, m^2 (q.q') for S = III."""
    if S == 1:
        return mdot(q, a) * mdot(qp, b)
    if S == 2:
        return mdot(q, b) * mdot(qp, a)
    return m * m * mdot(q, qp)


def brute_nes_avg(S, e, ep, E, x, m=M):
    """<M^S>_phi / k for nu(q) e(p) -> nu(q') e(p'), S = I: (q.p)(q'.p'), II: (q.p')(q'.p)."""
    q3, qp3, q, qp = _neutrinos(e, ep, x)
    k3 = q3 - qp3
    k = np.linalg.norm(k3)
    Ep = E + e - ep
    if E <= m or Ep <= m or k == 0:
        return None
    P, Pp = math.sqrt(E * E - m * m), math.sqrt(Ep * Ep - m * m)
    ca = (Pp * Pp - P * P - k * k) / (2 * P * k)
    if abs(ca) > 1:
        return None
    kh, e1, e2 = frame(k3)
    sa = math.sqrt(max(0.0, 1 - ca * ca))
    acc = 0.0
    for phi in 2 * np.pi * np.arange(NPHI) / NPHI:
        p = np.concatenate([[E], P * (ca * kh + sa * (np.cos(phi) * e1 + np.sin(phi) * e2))])
        pf = p + q - qp
        assert abs(mdot(p, p) - m * m) < 1e-9 * E * E and abs(mdot(pf, pf) - m * m) < 1e-9 * Ep * Ep
        acc += _structure(S, p, pf, q, qp, m)
    return acc / NPHI / k


def brute_pair_avg(S, e, ep, E, x, m=M):
    """<M^S>_phi / Q for nu(q) nubar(q') -> e-(p) e+(pbar), S = I: (q.pbar)(q'.p), II: (q.p)(q'.pbar)."""
    q3, qp3, q, qp = _neutrinos(e, ep, x)
    Q3 = q3 + qp3
    Q = np.linalg.norm(Q3)
    Eb = e + ep - E
    if E <= m or Eb <= m or Q == 0:
        return None
    P, Pb = math.sqrt(E * E - m * m), math.sqrt(Eb * Eb - m * m)
    ca = (P * P + Q * Q - Pb * Pb) / (2 * P * Q)
    if abs(ca) > 1:
        return None
    kh, e1, e2 = frame(Q3)
    sa = math.sqrt(max(0.0, 1 - ca * ca))
    acc = 0.0
    for phi in 2 * np.pi * np.arange(NPHI) / NPHI:
        p = np.concatenate([[E], P * (ca * kh + sa * (np.cos(phi) * e1 + np.sin(phi) * e2))])
        pb = q + qp - p
        assert abs(mdot(pb, pb) - m * m) < 1e-9 * Eb * Eb
        acc += _structure(S, pb, p, q, qp, m)
    return acc / NPHI / Q


def brute_h(avg, l, S, e, ep, E, pole):
    """Integral dx P_l(x) <M>/k over the open region; x = pole - pole u^2 removes the integrable
    1/k at the pole on the diagonal (the brute force is good to ~3e-8 there)."""
    def xof(u):
        return min(1.0, max(-1.0, pole - pole * u * u))

    def g(u):
        x = xof(u)
        v = avg(S, e, ep, E, x)
        return 0.0 if v is None else 2 * u * (v if l == 0 else x * v)

    def open_at(u):
        return avg(S, e, ep, E, xof(u)) is not None

    us = np.linspace(0, np.sqrt(2.0), 401)
    inside = np.array([open_at(u) for u in us])
    if not inside.any():
        return 0.0
    edges = [0.0, np.sqrt(2.0)]
    for a, b, ia, ib in zip(us[:-1], us[1:], inside[:-1], inside[1:]):
        if ia != ib:
            edges.append(so.brentq(lambda u: open_at(u) - 0.5, a, b, xtol=1e-15))
    tot = 0.0
    for a, b in zip(sorted(edges)[:-1], sorted(edges)[1:]):
        tot += si.quad(g, a, b, epsabs=0, epsrel=1e-11, limit=200)[0]
    return tot


# (eps, eps', E): far above the mass, at the MeV scale, just above the electron threshold,
# eps' << eps, and the near-diagonal case where the momentum-transfer interval starts near 0
CASES_NES = [(20.0, 10.0, 5.0), (2.0, 1.0, 0.8), (0.8, 0.5, 0.52), (5.0, 0.3, 1.0), (1.0, 2.0, 1.9),
             (3.0, 3.0, 0.7)]
CASES_PAIR = [(20.0, 10.0, 5.0), (2.0, 1.0, 0.8), (3.0, 0.5, 2.0), (1.0, 1.0, 1.0), (0.6, 0.6, 0.6),
              (0.7, 0.4, 0.53)]


@pytest.mark.parametrize("e,ep,E", CASES_NES)
@pytest.mark.parametrize("l", [0, 1])
@pytest.mark.parametrize("S", [1, 2, 3])
def test_nes_vs_brute_force(e, ep, E, l, S):
    ref = brute_h(brute_nes_avg, l, S, e, ep, E, 1.0)
    got = float(massive.h_nes(l, S, e, ep, E))
    scale = abs(float(massive.h_nes(0, 1, e, ep, E)))
    assert scale > 0
    assert abs(got - ref) <= 5e-8 * scale, (got, ref)


@pytest.mark.parametrize("e,ep,E", CASES_PAIR)
@pytest.mark.parametrize("l", [0, 1])
@pytest.mark.parametrize("S", [1, 2, 3])
def test_pair_vs_brute_force(e, ep, E, l, S):
    ref = brute_h(brute_pair_avg, l, S, e, ep, E, -1.0)
    got = float(massive.h_pair(l, S, e, ep, E))
    scale = abs(float(massive.h_pair(0, 1, e, ep, E)))
    assert scale > 0
    assert abs(got - ref) <= 5e-8 * scale, (got, ref)


@pytest.mark.parametrize("e,ep,E", [(20.0, 10.0, 5.0), (20.0, 10.0, 15.0), (7.0, 7.0, 3.0), (3.0, 40.0, 45.0)])
def test_massless_limit(e, ep, E):
    for l in (0, 1):
        for S in (1, 2):
            for fm, fa in ((massive.h_nes, angular.h_nes), (massive.h_pair, angular.h_pair)):
                ref = float(fa(l, S, e, ep, E))
                scale = abs(float(fa(0, S, e, ep, E)))
                assert abs(float(fm(l, S, e, ep, E, m=1e-9)) - ref) <= 1e-12 * scale
        assert abs(float(massive.h_nes(l, 3, e, ep, E, m=1e-9))) <= 1e-15 * abs(float(angular.h_nes(0, 1, e, ep, E)))


def _vacuum_closed(e, ep, S, l):
    def g(x):
        s = 2 * e * ep * (1 - x)
        if s <= 4 * M * M:
            return 0.0
        b = math.sqrt(1 - 4 * M * M / s)
        v = b * s * s * (3 + b * b) / 48 if S in (1, 2) else b * M * M * s / 2
        return v * (x if l else 1.0)
    xmax = 1 - 2 * M * M / (e * ep)
    if xmax <= -1:
        return 0.0
    return si.quad(g, -1, xmax, epsabs=0, epsrel=1e-13, limit=200)[0]


@pytest.mark.parametrize("e,ep", [(10.0, 20.0), (0.6, 0.6), (1.0, 0.3), (0.9, 0.35), (5.0, 5.0), (0.5, 0.5)])
def test_vacuum_pair_cross_section(e, ep):
    """(0.5, 0.5): 4 eps eps' < 4 m^2, below threshold at every angle; (1.0, 0.3), (0.9, 0.35):
    the threshold cuts the angular range."""
    for S in (1, 2, 3):
        for l in (0, 1):
            f = lambda E: float(massive.h_pair(l, S, e, ep, E))
            lo, hi = M, e + ep - M
            if hi <= lo:
                assert _vacuum_closed(e, ep, S, l) == 0.0
                continue
            pts = np.linspace(lo, hi, 9)
            got = sum(si.quad(f, a, b, epsabs=0, epsrel=1e-12, limit=400)[0] for a, b in zip(pts[:-1], pts[1:]))
            ref = _vacuum_closed(e, ep, S, l)
            if ref == 0.0:
                assert got == 0.0
            else:
                assert abs(got - ref) <= 1e-11 * abs(ref), (S, l, got, ref)


@pytest.mark.parametrize("e,T", [(5.0, 1.0), (2.0, 0.5), (0.8, 0.2), (1.2, 0.9)])
def test_electron_at_rest(e, T):
    ep = e - T
    E = M * (1 + 1e-12)
    H = [float(massive.h_nes(0, S, e, ep, E)) for S in (1, 2, 3)]
    assert H[0] > 0
    assert abs(H[1] / H[0] - (ep / e) ** 2) <= 1e-5 * (ep / e) ** 2
    assert abs(H[2] / H[0] - M * T / e ** 2) <= 1e-5 * (M * T / e ** 2)


@pytest.mark.parametrize("e,ep,E", [(2.0, 1.0, 0.8), (0.8, 0.5, 0.52), (5.0, 0.3, 1.0), (3.0, 3.0, 0.7)])
def test_time_reversal_and_transpose(e, ep, E):
    for l in (0, 1):
        for S in (1, 2, 3):
            a = float(massive.h_nes(l, S, e, ep, E))
            b = float(massive.h_nes(l, S, ep, e, E + e - ep))
            assert abs(a - b) <= 1e-13 * abs(float(massive.h_nes(0, 1, e, ep, E)))
        for S, St in ((1, 2), (2, 1), (3, 3)):
            a = float(massive.h_pair(l, S, e, ep, E))
            b = float(massive.h_pair(l, St, ep, e, E))
            assert abs(a - b) <= 1e-13 * abs(float(massive.h_pair(0, 1, e, ep, E)))


def test_thresholds_close():
    # electron below its rest energy; final electron below it; pair below 2m
    assert float(massive.h_nes(0, 1, 2.0, 1.0, 0.5 * M)) == 0.0
    assert float(massive.h_nes(0, 1, 1.0, 2.0, 1.5 * M)) == 0.0      # E' = E - 1 < m
    assert float(massive.h_pair(0, 1, 0.4, 0.5, 0.45)) == 0.0        # eps + eps' < 2m
