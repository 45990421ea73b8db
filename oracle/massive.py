"""Angular weights with the electron mass (oracle; test infrastructure only).

The massless weights (oracle.angular) drop the electron mass m. With it, for neutrino
momenta q, q' (eps, eps') and an electron of energy E >= m, momentum P = sqrt(E^2 - m^2), the
spin-summed V-A matrix element gains a third structure,
  scattering nu e -> nu e:   32 G_F^2 [beta_I (q.p)(q'.p') + beta_II (q.p')(q'.p) - beta_III m^2 (q.q')],
  pair nu nubar -> e- e+:    32 G_F^2 [beta_I (q.pbar)(q'.p) + beta_II (q.p)(q'.pbar) + beta_III m^2 (q.q')],
with beta_III = C_V^2 - C_A^2 (the pair's sign follows from crossing two fermions into the
final state, which flips q'), and the kinematics change: the electron's spatial momentum is
P, not E. The phase-space reduction int d^3p/(2E) d^3p'/(2E') delta^4 = int dE dphi / (4 k)
is unchanged, with E >= m.

  H^S_l(eps, eps', E) = 1/(eps eps') Integral dk P_l(x(k)) <M^S>_phi, S = I, II, III,

Scattering, k = |q - q'|, omega = eps - eps', E' = E + omega >= m, P' = sqrt(E'^2 - m^2),
Q^2 = k^2 - omega^2 = 2 q.q':
  cos(alpha) = (2 E omega - Q^2) / (2 P k)                [p relative to k; from |p + k| = P']
  cos(beta) = (eps - eps' x)/k, cos(beta') = (eps x - eps')/k, sin b sin b' = eps eps'(1-x^2)/k^2
  <q.p> = eps (E - P cos b cos a), <q'.p> = eps' (E - P cos b' cos a),
  <(q.p)(q'.p)> = eps eps' [E^2 - E P (cos b + cos b') cos a
                            + P^2 (cos b cos b' cos^2 a + 1/2 sin b sin b' (1 - cos^2 a))],
  M^I = <(q.p)(q'.p)> + Q^2/2 <q.p>, M^II = <(q.p)(q'.p)> - Q^2/2 <q'.p>, M^III = m^2 Q^2/2,
  k in [max(|omega|, |P - P'|), min(eps + eps', P + P')].
Pair, Q = |q + q'|, w = eps + eps', Ebar = w - E >= m, Pbar = sqrt(Ebar^2 - m^2),
s = w^2 - Q^2 = 2 q.q':
  cos(alpha) = (Q^2 + P^2 - Pbar^2) / (2 Q P),
  cos(beta) = (eps + eps' x)/Q, cos(beta') = (eps' + eps x)/Q, the sin b sin b' term with the
  opposite sign (q, q' on opposite sides of Q),
  M^I = s/2 <q'.p> - <(q.p)(q'.p)>, M^II = s/2 <q.p> - <(q.p)(q'.p)>, M^III = m^2 s/2,
  Q in [max(|eps - eps'|, |P - Pbar|), min(w, P + Pbar)].
At m = 0 these are the massless weights (P = E), and M^III vanishes.

Evaluation: the k-integrand is a Laurent polynomial in k with even powers only (-4 .. 8 with
P_1), so there is no logarithm; the oracle integrates it by Gauss-Legendre in k, 12 nodes on
each of a graded set of subintervals: [k0, k1] is cut at k0 + L 2^-j, j = 1 .. J (L = k1 - k0),
with J the smallest level at which L 2^-J <= k0 (at most 60). Every subinterval then lies at
least its own length away from k = 0, the integrand's only singular point, so the rule is exact
for the polynomial part and accurate to ~1e-18 relative for the negative powers (Bernstein
ellipse radius >= 3 + 2 sqrt 2). Near-diagonal cases, where k0 -> 0 with nonzero k^-2 and k^-4
coefficients, are why a single interval would not do. Every function accepts arrays; E below
its threshold (m, or E' < m) gives 0.
"""
import numpy as np

ME = 0.51099895   # electron mass, MeV

_X, _W = np.polynomial.legendre.leggauss(12)
_MAX_LEVEL = 60


def _legendre_factor(l, x):
    return 1.0 if l == 0 else x


def _nes_integrand(l, S, e, ep, E, P, m, k):
    om = e - ep
    Q2 = (k - np.abs(om)) * (k + np.abs(om))
    one_m_x = Q2 / (2 * e * ep)
    one_p_x = ((e + ep) - k) * ((e + ep) + k) / (2 * e * ep)
    x = 1 - one_m_x
    ca = (2 * E * om - Q2) / (2 * P * k)
    cb = (e * e - ep * ep + k * k) / (2 * e * k)
    cbp = (e * e - ep * ep - k * k) / (2 * ep * k)
    sbsb = e * ep * one_m_x * one_p_x / (k * k)
    qp = e * (E - P * cb * ca)
    qpp = ep * (E - P * cbp * ca)
    qqp = e * ep * (E * E - E * P * (cb + cbp) * ca + P * P * (cb * cbp * ca * ca + 0.5 * sbsb * (1 - ca * ca)))
    if S == 1:
        M = qqp + 0.5 * Q2 * qp
    elif S == 2:
        M = qqp - 0.5 * Q2 * qpp
    else:
        M = m * m * 0.5 * Q2
    return _legendre_factor(l, x) * M / (e * ep)


def _pair_integrand(l, S, e, ep, E, P, Pb, m, k):
    w = e + ep
    s = (w - k) * (w + k)
    one_m_x = s / (2 * e * ep)
    d = np.abs(e - ep)
    one_p_x = (k - d) * (k + d) / (2 * e * ep)
    x = 1 - one_m_x
    ca = (k * k + P * P - Pb * Pb) / (2 * k * P)
    cb = (e * e - ep * ep + k * k) / (2 * e * k)
    cbp = (ep * ep - e * e + k * k) / (2 * ep * k)
    sbsb = e * ep * one_m_x * one_p_x / (k * k)
    qp = e * (E - P * cb * ca)
    qpp = ep * (E - P * cbp * ca)
    qqp = e * ep * (E * E - E * P * (cb + cbp) * ca + P * P * (cb * cbp * ca * ca - 0.5 * sbsb * (1 - ca * ca)))
    if S == 1:
        M = 0.5 * s * qpp - qqp
    elif S == 2:
        M = 0.5 * s * qp - qqp
    else:
        M = m * m * 0.5 * s
    return _legendre_factor(l, x) * M / (e * ep)


def _rule(fn, a, b):
    half, mid = 0.5 * (b - a), 0.5 * (b + a)
    out = 0.0
    for xg, wg in zip(_X, _W):
        out = out + wg * half * fn(mid + half * xg)
    return out


def _gauss(fn, k0, k1):
    """Integral of fn(k) over [k0, k1] (1-D arrays, k1 > k0 >= 0) on the graded subintervals.
    fn(k, sel) evaluates the integrand at k for the entries sel of the arrays."""
    L = k1 - k0
    with np.errstate(divide="ignore"):
        J = np.where(L <= k0, 0, np.ceil(np.log2(L / np.where(k0 > 0, k0, 1e-300))))
    J = np.clip(J, 0, _MAX_LEVEL).astype(int)
    out = np.zeros_like(k0)
    for j in range(int(J.max()) + 1 if J.size else 0):
        sel = np.nonzero(J >= j)[0]
        top = np.where(j == 0, 1.0, 2.0 ** -j)
        lo = np.where(J[sel] == j, 0.0, 0.5 * top)        # the last level keeps [k0, k0 + L 2^-J]
        a, b = k0[sel] + L[sel] * lo, k0[sel] + L[sel] * top
        out[sel] += _rule(lambda k: fn(k, sel), a, b)
    return out


def h_nes(l, S, e, ep, E, m=ME):
    """H^{N,S}_l with the electron mass, S = 1, 2, 3 (I, II, III); e, ep, E broadcast."""
    e, ep, E = np.broadcast_arrays(np.asarray(e, float), np.asarray(ep, float), np.asarray(E, float))
    om = e - ep
    Ep = E + om
    ok = (E > m) & (Ep > m)
    Es, Eps = np.where(ok, E, m + 1.0), np.where(ok, Ep, m + 1.0)
    P, Pp = np.sqrt((Es - m) * (Es + m)), np.sqrt((Eps - m) * (Eps + m))
    k0 = np.maximum(np.abs(om), np.abs(P - Pp))
    k1 = np.minimum(e + ep, P + Pp)
    ok = ok & (k1 > k0)
    k0s, k1s = np.where(ok, k0, 1.0).ravel(), np.where(ok, k1, 2.0).ravel()
    a = [v.ravel() for v in (e, ep, Es, P)]
    val = _gauss(lambda k, s: _nes_integrand(l, S, a[0][s], a[1][s], a[2][s], a[3][s], m, k), k0s, k1s)
    return np.where(ok, val.reshape(ok.shape), 0.0)


def h_pair(l, S, e, ep, E, m=ME):
    """H^{P,S}_l with the electron mass for nu(eps) nubar(eps') -> e-(E) e+(eps + eps' - E)."""
    e, ep, E = np.broadcast_arrays(np.asarray(e, float), np.asarray(ep, float), np.asarray(E, float))
    w = e + ep
    Eb = w - E
    ok = (E > m) & (Eb > m)
    Es, Ebs = np.where(ok, E, m + 1.0), np.where(ok, Eb, m + 1.0)
    P, Pb = np.sqrt((Es - m) * (Es + m)), np.sqrt((Ebs - m) * (Ebs + m))
    k0 = np.maximum(np.abs(e - ep), np.abs(P - Pb))
    k1 = np.minimum(w, P + Pb)
    ok = ok & (k1 > k0)
    k0s, k1s = np.where(ok, k0, 1.0).ravel(), np.where(ok, k1, 2.0).ravel()
    a = [v.ravel() for v in (e, ep, Es, P, Pb)]
    val = _gauss(lambda k, s: _pair_integrand(l, S, a[0][s], a[1][s], a[2][s], a[3][s], a[4][s], m, k), k0s, k1s)
    return np.where(ok, val.reshape(ok.shape), 0.0)


# ---------------------------------------------------------------------------------------
# Rates with the electron mass: the quadrature rule over the electron's total energy E and
# the task quadratures, in the layout of oracle.rates (completion, species sums and the
# contraction are that module's, with a third structure).
#
# Chemical potentials include the rest mass: F(E) = 1/(exp((E - mu)/T) + 1) for electrons of
# total energy E >= m, positrons at -mu.
#
# Rule, scattering task eps_i >= eps_j (omega = eps_i - eps_j >= 0). The weights are smooth in
# E except at the electron threshold E = m, where they grow like sqrt(E - m), and at one
# kink E_k >= m: the root of P + P' = eps_i + eps_j (the upper end of the momentum-transfer
# range switches from P + P' to eps_i + eps_j there, or the range opens there when
# P' - P > eps_i + eps_j at threshold; both conditions reduce to the same quadratic),
#   E_k = (sqrt(omega^2 + 4 eps_i eps_j + w^2 m^2/(eps_i eps_j)) - omega)/2,  w = eps_i + eps_j,
# which is eps_j at m = 0. Breakpoints as in the massless rule with 0 -> m and eps_j -> E_k:
#   b = sort(m, max(m, mu - omega), max(m, mu), min(E_k, max(m, mu) + KAPPA T));
# three Gauss-Legendre panels in s on [m, b_3], E = m + (b_3 - m) s^2 (so sqrt(E - m) is
# linear in s), and the Gauss-Laguerre tail E = b_3 + T x; n/4 nodes each.
# Rule, pair task (w = eps_i + eps_j): the weights vanish unless eps_i eps_j > m^2 (s_max =
# 4 eps_i eps_j above 4 m^2); they are smooth in E on [m, w - m] except at both thresholds
# (sqrt) and at E = (w -+ y)/2, y = |eps_i - eps_j| sqrt(1 - m^2/(eps_i eps_j)), where
# |P - Pbar| = |eps_i - eps_j| (or P + Pbar = |eps_i - eps_j|, the edge of the support).
#   b = sort(m, (w - y)/2, (w + y)/2, clip(mu, m, w - m), w - m): four Gauss-Legendre panels
# in theta, E = m + (w - 2m) sin^2(pi theta / 2), which is quadratic at both ends. Tasks
# (i, j) and (j, i) get identical nodes. Without support every weight is 0.
# ---------------------------------------------------------------------------------------
from . import physics as _phys          # noqa: E402
from . import rates as _rates           # noqa: E402
from .rule import KAPPA as _KAPPA, gauss_laguerre_scaled as _glag, gauss_legendre01 as _gl01   # noqa: E402


def nes_kink(e, ep, m=ME):
    """E_k >= m of the scattering task (e >= ep)."""
    e, ep = np.asarray(e, float), np.asarray(ep, float)
    om, w = e - ep, e + ep
    Ek = 0.5 * (np.sqrt(om * om + 4.0 * e * ep + w * w * m * m / (e * ep)) - om)
    return np.maximum(Ek, m)


def pair_kinks(e, ep, m=ME):
    """((w - y)/2, (w + y)/2) and the support flag eps_i eps_j > m^2 and w > 2m."""
    e, ep = np.asarray(e, float), np.asarray(ep, float)
    w = e + ep
    ok = (e * ep > m * m) & (w > 2 * m)
    y = np.abs(e - ep) * np.sqrt(np.where(ok, 1.0 - m * m / np.where(ok, e * ep, 1.0), 0.0))
    return 0.5 * (w - y), 0.5 * (w + y), ok


def _panels_mapped(bounds, m4, emap, dmap):
    """Gauss-Legendre panels in a map variable v between consecutive breakpoints (given in
    v); E = emap(v), W = w dv dE/dv."""
    t, wt = _gl01(m4)
    a = bounds[..., :-1, None]
    L = bounds[..., 1:, None] - a
    v = a + L * t
    E = emap(v)
    W = L * wt * dmap(v)
    return E.reshape(E.shape[:-2] + (-1,)), W.reshape(W.shape[:-2] + (-1,))


def nes_nodes(eps_i, eps_j, T, mu, n, m=ME):
    """(E, W) [..., n] of the scattering task eps_i >= eps_j with the electron mass."""
    eps_i, eps_j, T, mu = np.broadcast_arrays(np.asarray(eps_i, float), np.asarray(eps_j, float),
                                              np.asarray(T, float), np.asarray(mu, float))
    if n % 4:
        raise ValueError("bad node count")
    m4 = n // 4
    om = eps_i - eps_j
    u = np.maximum(m, mu)
    b = np.sort(np.stack([np.full_like(mu, m), np.maximum(m, mu - om), u,
                          np.minimum(nes_kink(eps_i, eps_j, m), u + _KAPPA * T)], axis=-1), axis=-1)
    L = (b[..., 3] - m)[..., None, None]
    Ls = np.where(L > 0, L, 1.0)
    s = np.sqrt(np.maximum(b - m, 0.0) / Ls[..., 0])
    E1, W1 = _panels_mapped(s, m4, lambda v: m + L * v * v, lambda v: 2.0 * L * v)
    x, wx = _glag(m4)
    E2 = b[..., 3:4] + T[..., None] * x
    W2 = T[..., None] * wx + 0.0 * E2
    return np.concatenate([E1, E2], axis=-1), np.concatenate([W1, W2], axis=-1)


def pair_nodes(eps_i, eps_j, T, mu, n, m=ME):
    """(E, W) [..., n] of the pair task (eps_i, eps_j) with the electron mass."""
    eps_i, eps_j, T, mu = np.broadcast_arrays(np.asarray(eps_i, float), np.asarray(eps_j, float),
                                              np.asarray(T, float), np.asarray(mu, float))
    if n % 4:
        raise ValueError("bad node count")
    w = eps_i + eps_j
    lo, hi, ok = pair_kinks(eps_i, eps_j, m)
    span = np.where(ok, w - 2 * m, 1.0)
    top = m + span
    c = np.clip(mu, m, top)
    b = np.sort(np.stack([np.full_like(mu, m), np.clip(lo, m, top), np.clip(hi, m, top), c, top], axis=-1), axis=-1)
    th = np.arccos(np.clip(1.0 - 2.0 * (b - m) / span[..., None], -1.0, 1.0)) / np.pi
    sp_ = span[..., None, None]
    E, W = _panels_mapped(th, n // 4, lambda v: m + sp_ * np.sin(0.5 * np.pi * v) ** 2,
                          lambda v: sp_ * 0.5 * np.pi * np.sin(np.pi * v))
    return E, np.where(ok[..., None], W, 0.0)


def scattering_quadrature(eps, T, mu, opts, absolute=False, m=ME):
    """q[z, t, S, l], S = I, II, III, tasks t = (i >= j); the third structure carries the minus
    sign it has in the scattering matrix element, so the species sum is sum_S beta_S q_S."""
    ii, jj = _rates.nes_tasks(eps.shape[0])
    ei = eps[ii][None, :]
    ej = eps[jj][None, :]
    Tz = T[:, None]
    muz = mu[:, None]
    E, W = nes_nodes(ei, ej, Tz, muz, opts.nquad, m)
    delta = (ei - ej)[..., None]
    B = _rates.fermi(E, muz[..., None], Tz[..., None]) * _rates.one_minus_fermi(E + delta, muz[..., None], Tz[..., None])
    pref = _phys.G_F ** 2 / (np.pi * ei * ej)
    out = []
    for S, sign in ((1, 1.0), (2, 1.0), (3, -1.0)):
        row = []
        for l in (0, 1):
            H = h_nes(l, S, ei[..., None], ej[..., None], E, m)
            H = np.abs(H) if absolute else sign * H
            row.append(pref * np.sum(W * B * H, axis=-1))
        out.append(np.stack(row, axis=-1))
    return np.stack(out, axis=-2)


def pair_quadrature(eps, T, mu, opts, absolute=False, m=ME):
    """(A, A3) [z, i, j, l]: structure I of the pair (i, j) (structure II is A of (j, i)) and
    the symmetric third structure, with the plus sign it has in the pair matrix element."""
    ne = eps.shape[0]
    ei = eps[:, None][None]
    ej = eps[None, :][None]
    Tz = T[:, None, None]
    muz = mu[:, None, None]
    E, W = pair_nodes(ei, ej, Tz, muz, opts.nquad, m)
    w = (ei + ej)[..., None]
    B = _rates.one_minus_fermi(E, muz[..., None], Tz[..., None]) * \
        _rates.one_minus_fermi_positron(w - E, muz[..., None], Tz[..., None])
    pref = _phys.G_F ** 2 / (np.pi * ei * ej)
    res = []
    for S in (1, 3):
        out = []
        for l in (0, 1):
            H = h_pair(l, S, ei[..., None], ej[..., None], E, m)
            H = np.abs(H) if absolute else H
            out.append(pref * np.sum(W * B * H, axis=-1))
        res.append(np.stack(out, axis=-1).reshape(T.shape[0], ne, ne, 2))
    return res[0], res[1]


def task_quadratures(eps, T, eta_e, opts, absolute=False, m=ME):
    """The massive counterpart of oracle.rates.task_quadratures: "nes"/"nps" q[z, t, 3, l],
    "pair" A and "pair3" A3 [z, i, j, l]."""
    eps = np.asarray(eps, dtype=float)
    T = np.asarray(T, dtype=float)
    mu = np.asarray(eta_e, dtype=float) * T
    out = {}
    for bit, name, mm in ((_rates.PROC_NES, "nes", mu), (_rates.PROC_NPS, "nps", -mu)):
        if opts.processes & bit:
            out[name] = scattering_quadrature(eps, T, mm, opts, absolute, m)
    if opts.processes & _rates.PROC_PAIR:
        out["pair"], out["pair3"] = pair_quadrature(eps, T, mu, opts, absolute, m)
    return out
