"""Pins for the oracle's angular weights H (oracle.angular).

* brute force: explicit four-vectors for the neutrinos and the electron, the azimuthal
  average taken numerically on a uniform phi grid (exact for the degree-2 trigonometric
  polynomials involved), the kinematic range found numerically (|cos alpha| <= 1), and the
  momentum-transfer integral done by adaptive quadrature in x = cos(q, q'); l = 0 and 1, on
  both of the oracle's routes (exact Laurent terms, and the direct integrand on short
  momentum-transfer intervals);
* closed-form l = 0 pieces for eps > eps' (independent symbolic integration);
* time reversal H^N(eps', eps, E + eps - eps') = H^N(eps, eps', E) and pair transposition
  H^{P,II}(eps, eps', E) = H^{P,I}(eps', eps, E).
"""
import numpy as np
import pytest
import scipy.integrate as si
import scipy.optimize as so

from oracle.angular import h_nes, h_pair


def mdot(a, b):
    return a[0] * b[0] - np.dot(a[1:], b[1:])


def frame(axis):
    k = axis / np.linalg.norm(axis)
    t = np.array([1.0, 0.0, 0.0]) if abs(k[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(k, t)
    e1 /= np.linalg.norm(e1)
    return k, e1, np.cross(k, e1)


NPHI = 16


def brute_nes_avg(S, e, ep, E, x):
    """<M^S>_phi / k for scattering at fixed cos(q, q') = x, or None if kinematically closed."""
    q3 = e * np.array([0.0, 0.0, 1.0])
    qp3 = ep * np.array([np.sqrt(1 - x * x), 0.0, x])
    k3 = q3 - qp3
    k = np.linalg.norm(k3)
    Ep = E + e - ep
    if Ep < 0 or k == 0:
        return None
    ca = (Ep * Ep - E * E - k * k) / (2 * E * k)
    if abs(ca) > 1:
        return None
    kh, e1, e2 = frame(k3)
    sa = np.sqrt(max(0.0, 1 - ca * ca))
    q = np.concatenate([[e], q3])
    qp = np.concatenate([[ep], qp3])
    acc = 0.0
    for phi in 2 * np.pi * np.arange(NPHI) / NPHI:
        p3 = E * (ca * kh + sa * (np.cos(phi) * e1 + np.sin(phi) * e2))
        p = np.concatenate([[E], p3])
        pf = p + q - qp
        assert abs(mdot(pf, pf)) < 1e-8 * max(1.0, E * E)
        acc += mdot(q, p) * mdot(qp, pf) if S == 1 else mdot(q, pf) * mdot(qp, p)
    return acc / NPHI / k


def brute_pair_avg(S, e, ep, E, x):
    q3 = e * np.array([0.0, 0.0, 1.0])
    qp3 = ep * np.array([np.sqrt(1 - x * x), 0.0, x])
    Q3 = q3 + qp3
    Q = np.linalg.norm(Q3)
    Eb = e + ep - E
    if Eb < 0 or E < 0 or Q == 0:
        return None
    ca = (E * E + Q * Q - Eb * Eb) / (2 * E * Q)
    if abs(ca) > 1:
        return None
    kh, e1, e2 = frame(Q3)
    sa = np.sqrt(max(0.0, 1 - ca * ca))
    q = np.concatenate([[e], q3])
    qp = np.concatenate([[ep], qp3])
    acc = 0.0
    for phi in 2 * np.pi * np.arange(NPHI) / NPHI:
        p = np.concatenate([[E], E * (ca * kh + sa * (np.cos(phi) * e1 + np.sin(phi) * e2))])
        pb = q + qp - p
        assert abs(mdot(pb, pb)) < 1e-8 * max(1.0, E * E)
        acc += mdot(q, pb) * mdot(qp, p) if S == 1 else mdot(q, p) * mdot(qp, pb)
    return acc / NPHI / Q


def brute_h(avg, l, S, e, ep, E, pole):
    """H = Integral dx P_l(x) <M>/k over the open kinematic region (found by bisection).

    The momentum transfer vanishes at x = pole (+1 scattering, -1 pair) on the diagonal;
    x = pole - pole u^2 removes that integrable 1/k singularity."""
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
    edges = sorted(edges)
    tot = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        tot += si.quad(g, a, b, epsabs=0, epsrel=1e-11, limit=200)[0]
    return tot


CASES_NES = [(20.0, 10.0, 5.0), (20.0, 10.0, 15.0), (10.0, 20.0, 15.0), (7.0, 7.0, 3.0), (3.0, 40.0, 45.0),
             (33.0, 4.5, 80.0)]
CASES_PAIR = [(20.0, 10.0, 5.0), (20.0, 10.0, 15.0), (20.0, 10.0, 25.0), (6.0, 6.0, 4.0), (3.0, 50.0, 30.0)]
# Short momentum-transfer intervals (k1 - k0 <= k0), where the oracle integrates the directly
# evaluated integrand instead of the exact Laurent terms: E / eps' = 0.015, eps' / eps = 0.015,
# eps << eps' just above threshold; pair with eps' << eps and with E near either end.
CASES_NES_SHORT = [(20.0, 10.0, 0.15), (100.0, 1.5, 30.0), (1.5, 100.0, 98.7)]
CASES_PAIR_SHORT = [(100.0, 1.5, 30.0), (20.0, 10.0, 0.3), (20.0, 10.0, 29.7)]


@pytest.mark.parametrize("e,ep,E", CASES_NES + CASES_NES_SHORT)
@pytest.mark.parametrize("l", [0, 1])
@pytest.mark.parametrize("S", [1, 2])
def test_nes_vs_brute_force(e, ep, E, l, S):
    ref = brute_h(brute_nes_avg, l, S, e, ep, E, 1.0)
    got = float(h_nes(l, S, e, ep, E))
    scale = abs(float(h_nes(0, S, e, ep, E)))
    assert abs(got - ref) <= 5e-8 * scale, (got, ref)


@pytest.mark.parametrize("e,ep,E", CASES_PAIR + CASES_PAIR_SHORT)
@pytest.mark.parametrize("l", [0, 1])
@pytest.mark.parametrize("S", [1, 2])
def test_pair_vs_brute_force(e, ep, E, l, S):
    ref = brute_h(brute_pair_avg, l, S, e, ep, E, -1.0)
    got = float(h_pair(l, S, e, ep, E))
    scale = abs(float(h_pair(0, S, e, ep, E)))
    assert abs(got - ref) <= 5e-8 * scale, (got, ref)


def test_closed_form_l0_pieces():
    """eps > eps': l = 0 pieces obtained by symbolic integration, written out."""
    e, ep = 23.0, 9.0
    for E in np.linspace(0.3, 60.0, 37):
        if E < ep:
            n1 = 4 * E ** 3 * (E ** 2 + 5 * E * e + 10 * e ** 2) / (15 * e * ep)
            n2 = 4 * E ** 3 * (E ** 2 - 5 * E * ep + 10 * ep ** 2) / (15 * e * ep)
        else:
            n1 = 4 * ep ** 2 * (10 * E ** 2 + 20 * E * e - 15 * E * ep + 10 * e ** 2 - 15 * e * ep + 6 * ep ** 2) / (15 * e)
            n2 = 4 * ep ** 2 * (10 * E ** 2 - 5 * E * ep + ep ** 2) / (15 * e)
        assert np.isclose(h_nes(0, 1, e, ep, E), n1, rtol=1e-11, atol=0)
        assert np.isclose(h_nes(0, 2, e, ep, E), n2, rtol=1e-11, atol=0)
        if E < e + ep:
            if E < ep:
                p1 = 4 * E ** 3 * (E ** 2 - 5 * E * ep + 10 * ep ** 2) / (15 * e * ep)
            elif E < e:
                p1 = 4 * ep ** 2 * (10 * E ** 2 - 5 * E * ep + ep ** 2) / (15 * e)
            else:
                p1 = -4 * (E - e - ep) ** 3 * (E ** 2 + 3 * E * e - 2 * E * ep + 6 * e ** 2 - 3 * e * ep + ep ** 2) / (15 * e * ep)
            assert np.isclose(h_pair(0, 1, e, ep, E), p1, rtol=1e-9, atol=1e-12 * (e * ep) ** 2)
        else:
            assert h_pair(0, 1, e, ep, E) == 0.0


def test_closed_form_diagonal():
    e = 7.0
    for E in (0.5, 3.0, 6.9):
        assert np.isclose(h_nes(0, 1, e, e, E), 4 * E ** 3 * (E ** 2 + 5 * E * e + 10 * e ** 2) / (15 * e * e), rtol=1e-12, atol=0)
        assert np.isclose(h_nes(0, 2, e, e, E), 4 * E ** 3 * (E ** 2 - 5 * E * e + 10 * e ** 2) / (15 * e * e), rtol=1e-12, atol=0)


def test_time_reversal_and_transpose():
    rng = np.random.default_rng(3)
    for _ in range(40):
        e, ep = rng.uniform(2, 200, 2)
        E = rng.uniform(max(0, ep - e) + 0.05, 300)
        for l in (0, 1):
            for S in (1, 2):
                a = h_nes(l, S, e, ep, E)
                b = h_nes(l, S, ep, e, E + e - ep)
                assert np.isclose(a, b, rtol=1e-9, atol=1e-12 * abs(h_nes(0, S, e, ep, E)))
                Ep = rng.uniform(0.05, e + ep - 0.05)
                assert np.isclose(h_pair(l, 2, e, ep, Ep), h_pair(l, 1, ep, e, Ep), rtol=1e-9,
                                  atol=1e-12 * (e * ep) ** 2)


def test_kinematic_zeros():
    assert h_nes(0, 1, 5.0, 20.0, 10.0) == 0.0     # E < eps' - eps: no allowed k
    assert h_pair(1, 1, 5.0, 20.0, 26.0) == 0.0    # E > eps + eps'
    assert h_pair(0, 2, 5.0, 20.0, 0.0) == 0.0
