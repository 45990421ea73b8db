"""Angular weights H of the neutrino-electron scattering and pair kernels (oracle).

Test infrastructure only. The paper names these interaction rates as a component of the
model's transport sources (Sect. 2.1) and prints no formula for them; what follows is the
standard weak-interaction matrix element for massless e+- reduced to one angle. Definition (massless e+-, momenta q, q' of the two neutrinos,
eps = |q|, eps' = |q'|, x = cos angle(q, q'), P_l Legendre polynomials):

  H_l^S(eps, eps', E) = 1/(eps eps') * Integral dk P_l(x(k)) <M^S>_phi(k, E)

where <.>_phi is the average over the electron's azimuth about the momentum-transfer axis
and the k-range is the kinematically allowed one. Every integrand is a Laurent polynomial
in k (powers -4..6, odd powers absent), so the integral is taken exactly, term by term.
Both kernels then read  Phi_l = G_F^2/(pi eps eps') Integral dE (blocking) sum_S beta_S H_l^S.

Scattering nu(q) e(p) -> nu(q') e(p'), k = |q - q'|, omega = eps - eps', Q^2 = k^2 - omega^2:
  cos(alpha) = (2 E omega - Q^2)/(2 E k)   [p relative to k]
  cos(beta) = (eps - eps' x)/k, cos(beta') = (eps x - eps')/k,
  sin(beta) sin(beta') = eps eps' (1 - x^2)/k^2   [q, q' on the same side of k]
  <q.p> = eps E (1 - cos b cos a), <q'.p> = eps' E (1 - cos b' cos a),
  <(q.p)(q'.p)> = eps eps' E^2 [1 - (cos b + cos b') cos a + cos b cos b' cos^2 a
                               + 1/2 sin b sin b' (1 - cos^2 a)],
  M^I = <(q.p)(q'.p)> + Q^2/2 <q.p>   (= (q.p)(q'.p')),
  M^II = <(q.p)(q'.p)> - Q^2/2 <q'.p> (= (q.p')(q'.p)),
  k in [|eps - eps'|, min(eps + eps', 2E + eps - eps')], empty unless E >= eps' - eps.
Pair nu(q) anti-nu(q') -> e-(p) e+(pbar), Q = |q + q'|, w = eps + eps', s = w^2 - Q^2:
  cos(alpha) = (2 w E - s)/(2 Q E), cos(beta) = (eps + eps' x)/Q, cos(beta') = (eps' + eps x)/Q,
  sin b sin b' = eps eps' (1 - x^2)/Q^2 with the OPPOSITE sign in the phi-average
  (q, q' on opposite sides of Q): ... - 1/2 sin b sin b' (1 - cos^2 a),
  M^I = s/2 <q'.p> - <(q.p)(q'.p)>  (= (q.pbar)(q'.p)),
  M^II = s/2 <q.p> - <(q.p)(q'.p)>  (= (q.p)(q'.pbar)),
  Q in [max(|eps - eps'|, |2E - w|), w],  0 <= E <= w.

Evaluation: where the k-interval is long (k1 - k0 > k0) the Laurent terms are integrated
exactly; where it is short (k1 - k0 <= k0, e.g. E << eps', or eps' << eps) those exact
terms cancel catastrophically, and the integrand -- evaluated directly from the cosines,
every difference of squares factored -- is integrated by 12-point Gauss-Legendre in k:
the polynomial part exactly, the negative powers to ~1e-18 relative (the only singularity,
k = 0, lies at least one interval length outside, Bernstein-ellipse radius >= 3 + 2 sqrt 2).

Pins (tests/test_oracle_angular.py): explicit-vector azimuthal average by brute force,
closed-form l = 0 pieces, vacuum pair integrals, time reversal and pair transposition.
All arithmetic accepts complex arrays (used for complex-step derivatives); decisions are
taken on real parts.
"""
import numpy as np


class Laurent:
    """Laurent polynomial in k with array coefficients: {power: ndarray}."""

    __slots__ = ("c",)

    def __init__(self, c):
        self.c = dict(c)

    @staticmethod
    def const(a):
        return Laurent({0: a})

    def __add__(self, o):
        o = o if isinstance(o, Laurent) else Laurent.const(o)
        out = dict(self.c)
        for p, v in o.c.items():
            out[p] = out[p] + v if p in out else v
        return Laurent(out)

    __radd__ = __add__

    def __neg__(self):
        return Laurent({p: -v for p, v in self.c.items()})

    def __sub__(self, o):
        return self + (-(o if isinstance(o, Laurent) else Laurent.const(o)))

    def __rsub__(self, o):
        return Laurent.const(o) - self

    def __mul__(self, o):
        if not isinstance(o, Laurent):
            return Laurent({p: v * o for p, v in self.c.items()})
        out = {}
        for p1, v1 in self.c.items():
            for p2, v2 in o.c.items():
                p = p1 + p2
                out[p] = out[p] + v1 * v2 if p in out else v1 * v2
        return Laurent(out)

    __rmul__ = __mul__

    def shift(self, n):
        """Multiply by k**n."""
        return Laurent({p + n: v for p, v in self.c.items()})

    def integrate(self, k0, k1):
        """Exact Integral_{k0}^{k1} sum_p c_p k^p dk (k0, k1 > 0 where the range is non-empty)."""
        tot = 0.0
        for p, v in self.c.items():
            if p == -1:
                tot = tot + v * (np.log(k1) - np.log(k0))
            else:
                tot = tot + v * (k1 ** (p + 1) - k0 ** (p + 1)) / (p + 1)
        return tot


K = Laurent({1: 1.0})


def _phi_average(e, ep, E, ca, cb, cbp, sbsb, sign):
    """<q.p>, <q'.p>, <(q.p)(q'.p)> from the direction cosines (sign = +1 same side, -1 opposite)."""
    qp = (1 - cb * ca) * (e * E)
    qpp = (1 - cbp * ca) * (ep * E)
    qqp = (1 - (cb + cbp) * ca + cb * cbp * ca * ca + sbsb * (1 - ca * ca) * (0.5 * sign)) * (e * ep * E * E)
    return qp, qpp, qqp


def _legendre(l, x):
    if l == 0:
        return Laurent.const(1.0)
    if l == 1:
        return x
    raise ValueError("only l = 0, 1")


def _real(a):
    return np.real(a)

_GL_X, _GL_W = np.polynomial.legendre.leggauss(12)


def _nes_direct(l, S, e, ep, E, k):
    """Scattering k-integrand P_l(x) <M^S>/(e e') at numeric k (arrays broadcast)."""
    om = e - ep
    aom = np.abs(om)
    Q2 = (k - aom) * (k + aom)                       # k^2 - omega^2
    one_m_x = Q2 / (2 * e * ep)
    one_p_x = ((e + ep) - k) * ((e + ep) + k) / (2 * e * ep)
    x = 1 - one_m_x
    ca = (2 * E * om - Q2) / (2 * E * k)
    cb = (e * e - ep * ep + k * k) / (2 * e * k)
    cbp = (e * e - ep * ep - k * k) / (2 * ep * k)
    sbsb = e * ep * one_m_x * one_p_x / (k * k)
    qp, qpp, qqp = _phi_average(e, ep, E, ca, cb, cbp, sbsb, +1.0)
    M = qqp + 0.5 * Q2 * qp if S == 1 else qqp - 0.5 * Q2 * qpp
    return (1.0 if l == 0 else x) * M / (e * ep)


def _pair_direct(l, S, e, ep, E, k):
    """Pair Q-integrand P_l(x) <M^S>/(e e') at numeric Q = k."""
    w = e + ep
    s = (w - k) * (w + k)
    one_m_x = s / (2 * e * ep)
    d = np.abs(e - ep)
    one_p_x = (k - d) * (k + d) / (2 * e * ep)
    x = 1 - one_m_x
    ca = (2 * w * E - s) / (2 * k * E)
    cb = (e * e - ep * ep + k * k) / (2 * e * k)
    cbp = (ep * ep - e * e + k * k) / (2 * ep * k)
    sbsb = e * ep * one_m_x * one_p_x / (k * k)
    qp, qpp, qqp = _phi_average(e, ep, E, ca, cb, cbp, sbsb, -1.0)
    M = 0.5 * s * qpp - qqp if S == 1 else 0.5 * s * qp - qqp
    return (1.0 if l == 0 else x) * M / (e * ep)


def _gauss_k(fn, l, S, e, ep, E, k0, k1):
    """12-point Gauss-Legendre integral of fn over k in [k0, k1] (1-D arrays)."""
    half = 0.5 * (k1 - k0)
    mid = 0.5 * (k1 + k0)
    k = mid[:, None] + half[:, None] * _GL_X[None, :]
    vals = fn(l, S, e[:, None], ep[:, None], E[:, None], k)
    return half * (vals @ _GL_W)


def _replace_short(tot, sel, fn, l, S, e, ep, E, k0, k1):
    """tot with the entries where sel holds recomputed by the Gauss route."""
    if not np.any(sel):
        return tot
    shape = np.broadcast(tot, e, ep, E, k0, k1).shape
    out = np.array(np.broadcast_to(tot, shape), dtype=np.result_type(tot, E, k1))
    out = np.atleast_1d(out)
    idx = np.nonzero(np.atleast_1d(np.broadcast_to(sel, shape)))
    pick = lambda a: np.atleast_1d(np.broadcast_to(a, shape))[idx]
    out[idx] = _gauss_k(fn, l, S, pick(e), pick(ep), pick(E), pick(k0), pick(k1))
    return out.reshape(shape)


def h_nes(l, S, e, ep, E):
    """H^{N,S}_l(eps, eps', E) for scattering nu(eps) -> nu(eps'); S in (1, 2) = (I, II).

    e, ep, E broadcast; e, ep real and positive, E may be complex (complex step)."""
    e, ep, E = np.broadcast_arrays(np.asarray(e, dtype=float), np.asarray(ep, dtype=float), np.asarray(E))
    ok = (_real(E) > 0) & (_real(E) >= ep - e)
    Es = np.where(ok, E, 1.0)
    wt = e - ep
    x = (K * K).__mul__(-1.0 / (2 * e * ep)) + (e * e + ep * ep) / (2 * e * ep)
    Q2 = K * K - wt * wt
    ca = (Q2 * -1.0 + 2 * Es * wt).shift(-1) * (1.0 / (2 * Es))
    cb = (x * -ep + e).shift(-1)
    cbp = (x * e - ep).shift(-1)
    sbsb = (1 - x * x).shift(-2) * (e * ep)
    qp, qpp, qqp = _phi_average(e, ep, Es, ca, cb, cbp, sbsb, +1.0)
    if S == 1:
        M = qqp + Q2 * qp * 0.5
    else:
        M = qqp - Q2 * qpp * 0.5
    integrand = _legendre(l, x) * M * (1.0 / (e * ep))
    k0 = np.abs(wt)
    k1 = np.where(_real(2 * Es + wt) < e + ep, 2 * Es + wt, e + ep)
    k0s = np.where(k0 > 0, k0, 1.0)
    # k0 = 0 only on the diagonal eps = eps', where every negative-power coefficient vanishes
    # identically (each carries a factor omega); integrate those terms from k0s and drop them.
    tot = 0.0
    for p, v in integrand.c.items():
        if p < -1:
            term = v * (k1 ** (p + 1) - k0s ** (p + 1)) / (p + 1)
            tot = tot + np.where(k0 > 0, term, 0.0)
        elif p == -1:
            raise AssertionError("log term in the scattering integrand")
        else:
            tot = tot + v * (k1 ** (p + 1) - k0 ** (p + 1)) / (p + 1)
    nonempty = ok & (_real(k1) > k0)
    short = _real(k1 - k0) <= k0
    tot = _replace_short(tot, short & nonempty, _nes_direct, l, S, e, ep, Es, k0, k1)
    return np.where(nonempty, tot, 0.0)


def h_pair(l, S, e, ep, E):
    """H^{P,S}_l(eps, eps', E) for annihilation nu(eps) anti-nu(eps') -> e-(E) e+(eps+eps'-E)."""
    e, ep, E = np.broadcast_arrays(np.asarray(e, dtype=float), np.asarray(ep, dtype=float), np.asarray(E))
    w = e + ep
    ok = (_real(E) > 0) & (_real(E) < w)
    Es = np.where(ok, E, 0.5 * w)
    x = (K * K).__mul__(1.0 / (2 * e * ep)) - (e * e + ep * ep) / (2 * e * ep)
    s = K * K * -1.0 + w * w
    ca = (s * -1.0 + 2 * w * Es).shift(-1) * (1.0 / (2 * Es))
    cb = (x * ep + e).shift(-1)
    cbp = (x * e + ep).shift(-1)
    sbsb = (1 - x * x).shift(-2) * (e * ep)
    qp, qpp, qqp = _phi_average(e, ep, Es, ca, cb, cbp, sbsb, -1.0)
    if S == 1:
        M = s * qpp * 0.5 - qqp
    else:
        M = s * qp * 0.5 - qqp
    integrand = _legendre(l, x) * M * (1.0 / (e * ep))
    a = np.where(_real(2 * Es - w) >= 0, 2 * Es - w, w - 2 * Es)   # |2E - w|, analytic in E
    k0 = np.where(_real(a) > np.abs(e - ep), a, np.abs(e - ep))
    k1 = w
    k0s = np.where(_real(k0) > 0, k0, 1.0)
    # k0 = 0 only where eps = eps' and E = w/2 at once; every negative-power coefficient
    # carries a factor (eps - eps') or (2E - w) and vanishes there: drop those terms.
    tot = 0.0
    for p, v in integrand.c.items():
        if p == -1:
            raise AssertionError("log term in the pair integrand")
        if p < -1:
            term = v * (k1 ** (p + 1) - k0s ** (p + 1)) / (p + 1)
            tot = tot + np.where(_real(k0) > 0, term, 0.0)
        else:
            tot = tot + v * (k1 ** (p + 1) - k0 ** (p + 1)) / (p + 1)
    short = _real(k1 - k0) <= _real(k0)
    tot = _replace_short(tot, short & ok, _pair_direct, l, S, e, ep, Es, k0, k1 + 0 * k0)
    return np.where(ok, tot, 0.0)
