"""Interaction kernels and emissivity/opacity contraction (oracle; test infrastructure only).

Steps, in the order the method takes them (FP64 throughout, complex-safe):

1. Scattering quadrature, tasks eps_i >= eps_j (down-scatter and diagonal):
     q_{l,S}(i,j) = G_F^2/(pi eps_i eps_j) sum_k W_k F(E_k) [1 - F(E_k + eps_i - eps_j)] H^{N,S}_l(eps_i, eps_j, E_k)
   with F(E) = 1/(exp((E - mu_e)/T) + 1) and the rule of ``oracle.rule``.
   Optional, scattering on positrons (process bit PROC_NPS): the same quadrature with the
   positron occupation Fbar(E) = F(E; -mu_e) in place of F, i.e. q evaluated at -mu_e, and
   the couplings of the antiparticle target, C_A -> -C_A, which swaps beta_I and beta_II.
2. Scattering completion (detailed balance, in/out symmetry), no quadrature:
     Phi_out(i,j) = q(i,j) for i >= j,  Phi_out(i,j) = exp(-(eps_j - eps_i)/T) q(j,i) for j > i,
     Phi_in(i,j) = Phi_out(j,i).
3. Pair quadrature, all (i,j):
     A_l(i,j) = G_F^2/(pi eps_i eps_j) sum_k W_k [1 - F(E_k)] [1 - Fbar(eps_i + eps_j - E_k)] H^{P,I}_l(eps_i, eps_j, E_k),
   Fbar(E) = 1/(exp((E + mu_e)/T) + 1);  Phi_a_I(i,j) = A(i,j), Phi_a_II(i,j) = A(j,i)
   (H^{P,II}(e, e', E) = H^{P,I}(e', e, E) and both tasks share nodes), production
   Phi_p = exp(-(eps_i + eps_j)/T) Phi_a.
4. Species: Phi^s = beta_I^s Phi_I + beta_II^s Phi_II  (``oracle.physics.couplings``).
5. Contraction with the P1 distribution f(mu) = f0 + 3 mu f1 of species s (partner sbar),
   c0 = 1/(4 pi^2 hbar c), bin volumes w_j:
     scattering: eta0 += c0 sum_j w_j Phi_in_0 f0(j)
                 chi0 += c0 sum_j w_j [Phi_in_0 f0(j) + Phi_out_0 (1 - f0(j))]
                 eta1 += c0 sum_j w_j Phi_in_1 f1(j)
                 chi1 += c0 sum_j w_j (Phi_in_1 - Phi_out_1) f1(j)
     pair:       eta0 += c0 sum_j w_j Phi_p_0 (1 - f0^sbar(j))
                 chi0 += c0 sum_j w_j [Phi_p_0 (1 - f0^sbar(j)) + Phi_a_0 f0^sbar(j)]
                 eta1 -= c0 sum_j w_j Phi_p_1 f1^sbar(j)
                 chi1 += c0 sum_j w_j (Phi_a_1 - Phi_p_1) f1^sbar(j)
   i.e. the collision term eta - chi f projected on the zeroth and first angular moments
   (the J, H moments of the paper's Eq. 1; intensity normalisation with (2 pi hbar c)^3,
   Sect. 2.1). A consumer forms S0 = eta0 - chi0 f0 - 3 chi1 f1, S1 = eta1 - chi1 f0 - chi0 f1.
Outputs eta[z][s][m][i], chi[z][s][m][i] in cm^-1.
6. Explicit Jacobian blocks (``jacobian``): the outputs are affine in f, so d out/d f is the
   coefficient of each f entry in step 5, block [s][p][o][i][j] for process p (scattering
   against f of s, pair against f of the partner) and output o = eta0, chi0, eta1, chi1 against
   f_{o//2}(j): the f-part of the Newton-Raphson Jacobian of the implicit solve (Sect. 2.1).

Pins: tests/test_oracle_rates.py (vacuum and non-degenerate closed forms, equilibrium null
test, continuous detailed balance by adaptive integration, linearity, couplings);
tests/test_oracle_jacobian.py (Jacobian blocks against the contraction and the complex-step
f-gradient).
"""
import dataclasses
import math

import numpy as np

from . import physics
from .angular import h_nes, h_pair
from .rule import RULE_PANEL, nes_nodes, pair_nodes

PROC_NES = 1
PROC_PAIR = 2
PROC_NPS = 4     # neutrino-positron scattering


@dataclasses.dataclass(frozen=True)
class Options:
    nquad: int = 48
    rule: str = RULE_PANEL
    processes: int = PROC_NES | PROC_PAIR
    sin2w: float = physics.SIN2W
    electron_mass: bool = False     # weights, rule and couplings with m_e (oracle.massive)


def _sigma(z):
    """Logistic 1/(1 + exp(-z)), overflow-free, decided on the real part."""
    with np.errstate(over="ignore", invalid="ignore"):
        pos = 1.0 / (1.0 + np.exp(-z))
        ez = np.exp(z)
        neg = ez / (1.0 + ez)
    return np.where(np.real(z) >= 0, pos, neg)


def fermi(E, mu, T):
    """Electron occupation 1/(exp((E - mu)/T) + 1)."""
    return _sigma((mu - E) / T)


def one_minus_fermi(E, mu, T):
    return _sigma((E - mu) / T)


def one_minus_fermi_positron(E, mu, T):
    """1 - 1/(exp((E + mu)/T) + 1) for positrons (chemical potential -mu)."""
    return _sigma((E + mu) / T)


def nes_tasks(ne):
    ii, jj = np.tril_indices(ne)
    return ii, jj


def scattering_quadrature(eps, T, mu, opts, absolute=False):
    """q[z, t, S, l] for tasks t = (i >= j) of ``nes_tasks``; S, l in {0, 1} (S index 0 = I).
    With ``absolute`` the angular weight enters as |H|: the sum of the absolute quadrature
    terms, the scale against which the rounding of a cancelling (l = 1) sum is judged."""
    ii, jj = nes_tasks(eps.shape[0])
    ei = eps[ii][None, :]
    ej = eps[jj][None, :]
    Tz = T[:, None]
    muz = mu[:, None]
    E, W = nes_nodes(ei, ej, Tz, muz, opts.nquad, opts.rule)
    delta = (ei - ej)[..., None]
    B = fermi(E, muz[..., None], Tz[..., None]) * one_minus_fermi(E + delta, muz[..., None], Tz[..., None])
    pref = physics.G_F ** 2 / (math.pi * ei * ej)
    out = []
    for S in (1, 2):
        row = []
        for l in (0, 1):
            H = h_nes(l, S, ei[..., None], ej[..., None], E)
            H = np.abs(H) if absolute else H
            row.append(pref * np.sum(W * B * H, axis=-1))
        out.append(np.stack(row, axis=-1))
    return np.stack(out, axis=-2)  # [z, t, S, l]


def pair_quadrature(eps, T, mu, opts, absolute=False):
    """A[z, i, j, l] for all bin pairs (``absolute``: |H|, as for the scattering quadrature)."""
    ne = eps.shape[0]
    ei = eps[:, None][None]
    ej = eps[None, :][None]
    Tz = T[:, None, None]
    muz = mu[:, None, None]
    E, W = pair_nodes(ei, ej, Tz, muz, opts.nquad)
    w = (ei + ej)[..., None]
    B = one_minus_fermi(E, muz[..., None], Tz[..., None]) * \
        one_minus_fermi_positron(w - E, muz[..., None], Tz[..., None])
    pref = physics.G_F ** 2 / (math.pi * ei * ej)
    out = []
    for l in (0, 1):
        H = h_pair(l, 1, ei[..., None], ej[..., None], E)
        H = np.abs(H) if absolute else H
        out.append(pref * np.sum(W * B * H, axis=-1))
    return np.stack(out, axis=-1).reshape(T.shape[0], ne, ne, 2)


def task_quadratures(eps, T, eta_e, opts, absolute=False):
    """Steps 1 and 3 only: the quadratures before completion, dict with "nes" / "nps"
    q[z, t, S, l] (tasks t = (i >= j)) and "pair" A[z, i, j, l]."""
    if opts.electron_mass:
        from . import massive
        return massive.task_quadratures(eps, T, eta_e, opts, absolute)
    eps = np.asarray(eps, dtype=float)
    T = np.asarray(T)
    mu = np.asarray(eta_e) * T
    out = {}
    for bit, name, m in ((PROC_NES, "nes", mu), (PROC_NPS, "nps", -mu)):
        if opts.processes & bit:
            out[name] = scattering_quadrature(eps, T, m, opts, absolute)
    if opts.processes & PROC_PAIR:
        out["pair"] = pair_quadrature(eps, T, mu, opts, absolute)
    return out


def complete(eps, T, quad):
    """Steps 2 and 3's completion from the quadratures of ``task_quadratures``: S-split
    kernels after completion, dict of arrays [z, i, j, S, l] (S index 0 = I)."""
    eps = np.asarray(eps, dtype=float)
    T = np.asarray(T)
    ne = eps.shape[0]
    out = {}
    for name in ("nes", "nps"):
        if name in quad:
            q = quad[name]
            nz = q.shape[0]
            ii, jj = nes_tasks(ne)
            full = np.zeros((nz, ne, ne) + q.shape[-2:], dtype=q.dtype)
            full[:, ii, jj] = q
            # up-scatter j > i from the down-scatter task (j, i): exp(-(eps_j - eps_i)/T); the
            # factor is formed for j > i only (elsewhere it would overflow at small T, unused)
            gap = np.maximum(eps[None, None, :] - eps[None, :, None], 0.0)
            up = np.exp(-gap / T[:, None, None])  # [z, i, j]
            upper = np.triu(np.ones((ne, ne), dtype=bool), 1)
            trans = np.swapaxes(full, 1, 2)
            phi_out = np.where(upper[None, :, :, None, None], up[..., None, None] * trans, full)
            out[name + "_out"] = phi_out
            out[name + "_in"] = np.swapaxes(phi_out, 1, 2)
    if "pair" in quad:
        A = quad["pair"]
        # [z, i, j, S, l]; with the electron mass the symmetric third structure follows
        phi_a = np.stack([A, np.swapaxes(A, 1, 2)] + ([quad["pair3"]] if "pair3" in quad else []), axis=-2)
        prod = np.exp(-(eps[None, :, None] + eps[None, None, :]) / T[:, None, None])
        out["pair_a"] = phi_a
        out["pair_p"] = prod[..., None, None] * phi_a
    return out


def zone_kernels(eps, T, eta_e, opts, absolute=False):
    """S-split kernels after completion: dict of arrays [z, i, j, S, l] (S index 0 = I)."""
    return complete(eps, T, task_quadratures(eps, T, eta_e, opts, absolute))


def _species(kern, beta):
    """sum_S beta_S kern[..., S, :] over the kernel's structures: (I, II), or (I, II, III)
    with the electron mass."""
    out = beta[0] * kern[..., 0, :]
    for S in range(1, kern.shape[-2]):
        out = out + beta[S] * kern[..., S, :]
    return out   # [z, i, j, l]


def scattering_kernels(kernels, b):
    """(Phi_in, Phi_out) [z, i, j, l] of one species with couplings b = (beta_I, beta_II[,
    beta_III]), summed over the scattering targets present: electrons with b, positrons with
    beta_I and beta_II swapped (C_A -> -C_A leaves beta_III = C_V^2 - C_A^2 alone)."""
    pin = pout = 0.0
    bp = (b[1], b[0]) + tuple(b[2:])
    if "nes_out" in kernels:
        pin = pin + _species(kernels["nes_in"], b)
        pout = pout + _species(kernels["nes_out"], b)
    if "nps_out" in kernels:
        pin = pin + _species(kernels["nps_in"], bp)
        pout = pout + _species(kernels["nps_out"], bp)
    return pin, pout


def has_scattering(kernels):
    return "nes_out" in kernels or "nps_out" in kernels


def contract(kernels, w, f, opts):
    """eta, chi [z, s, m, i] from completed kernels and f [z, s, m, j]."""
    w = np.asarray(w, dtype=float)
    cw = physics.C0 * w  # [j]
    nz, _, _, ne = f.shape
    dtype = np.result_type(f, *[k for k in kernels.values()])
    eta = np.zeros((nz, 3, 2, ne), dtype=dtype)
    chi = np.zeros((nz, 3, 2, ne), dtype=dtype)
    betas = physics.couplings(opts.sin2w, opts.electron_mass)
    for s in range(3):
        b = betas[s]
        if has_scattering(kernels):
            pin, pout = scattering_kernels(kernels, b)    # [z, i, j, l]
            f0 = f[:, s, 0, None, :] * cw
            g0 = (1.0 - f[:, s, 0, None, :]) * cw
            f1 = f[:, s, 1, None, :] * cw
            eta[:, s, 0] += np.sum(pin[..., 0] * f0, axis=-1)
            chi[:, s, 0] += np.sum(pin[..., 0] * f0 + pout[..., 0] * g0, axis=-1)
            eta[:, s, 1] += np.sum(pin[..., 1] * f1, axis=-1)
            chi[:, s, 1] += np.sum((pin[..., 1] - pout[..., 1]) * f1, axis=-1)
        if "pair_a" in kernels:
            sb = physics.PARTNER[s]
            pa = _species(kernels["pair_a"], b)
            pp = _species(kernels["pair_p"], b)
            f0 = f[:, sb, 0, None, :] * cw
            g0 = (1.0 - f[:, sb, 0, None, :]) * cw
            f1 = f[:, sb, 1, None, :] * cw
            eta[:, s, 0] += np.sum(pp[..., 0] * g0, axis=-1)
            chi[:, s, 0] += np.sum(pp[..., 0] * g0 + pa[..., 0] * f0, axis=-1)
            eta[:, s, 1] -= np.sum(pp[..., 1] * f1, axis=-1)
            chi[:, s, 1] += np.sum((pa[..., 1] - pp[..., 1]) * f1, axis=-1)
    return eta, chi


def contract_abs(kernels, w, f, opts):
    """Per-output sums of |terms| (A of the relative-error floor max(|y|, 1e-3 A))."""
    ak = {k: np.abs(v) for k, v in kernels.items()}
    w = np.asarray(w, dtype=float)
    cw = physics.C0 * w
    nz, _, _, ne = f.shape
    aeta = np.zeros((nz, 3, 2, ne))
    achi = np.zeros((nz, 3, 2, ne))
    betas = physics.couplings(opts.sin2w, opts.electron_mass)
    for s in range(3):
        b = tuple(abs(x) for x in betas[s])   # beta_III can be negative
        if has_scattering(ak):
            pin, pout = scattering_kernels(ak, b)
            f0 = f[:, s, 0, None, :] * cw
            g0 = np.abs(1.0 - f[:, s, 0, None, :]) * cw
            f1 = np.abs(f[:, s, 1, None, :]) * cw
            aeta[:, s, 0] += np.sum(pin[..., 0] * f0, axis=-1)
            achi[:, s, 0] += np.sum(pin[..., 0] * f0 + pout[..., 0] * g0, axis=-1)
            aeta[:, s, 1] += np.sum(pin[..., 1] * f1, axis=-1)
            achi[:, s, 1] += np.sum((pin[..., 1] + pout[..., 1]) * f1, axis=-1)
        if "pair_a" in ak:
            sb = physics.PARTNER[s]
            pa = _species(ak["pair_a"], b)
            pp = _species(ak["pair_p"], b)
            f0 = f[:, sb, 0, None, :] * cw
            g0 = np.abs(1.0 - f[:, sb, 0, None, :]) * cw
            f1 = np.abs(f[:, sb, 1, None, :]) * cw
            aeta[:, s, 0] += np.sum(pp[..., 0] * g0, axis=-1)
            achi[:, s, 0] += np.sum(pp[..., 0] * g0 + pa[..., 0] * f0, axis=-1)
            aeta[:, s, 1] += np.sum(pp[..., 1] * f1, axis=-1)
            achi[:, s, 1] += np.sum((pa[..., 1] + pp[..., 1]) * f1, axis=-1)
    return aeta, achi


PARTNER_OF_PROCESS = ((0, 1, 2), physics.PARTNER)   # species whose f a block multiplies


def jacobian_blocks(kernels, w, opts, absolute=False):
    """Explicit Jacobian blocks jac[z, s, p, o, i, j] = d out_o^s(i) / d f_m^{s'}(j).

    The outputs of step 5 are affine in f, so the derivative of each output with respect to
    one f entry is that entry's coefficient in step 5: p = 0 (scattering, s' = s) and p = 1
    (pair, s' = partner of s); o = eta0, chi0, eta1, chi1 with m = o // 2. These are the
    f-blocks of the Newton-Raphson Jacobian of the implicit transport step (Sect. 2.1).
    With ``absolute`` the entries are sums of |terms| instead (the error-floor scale).
    """
    k = {n: np.abs(v) for n, v in kernels.items()} if absolute else kernels
    cw = physics.C0 * np.asarray(w, dtype=float)          # [j]
    nz, ne = next(iter(k.values())).shape[:2]
    dtype = np.result_type(*[v for v in k.values()])
    jac = np.zeros((nz, 3, 2, 4, ne, ne), dtype=dtype)
    sgn = 1.0 if absolute else -1.0
    betas = physics.couplings(opts.sin2w, opts.electron_mass)
    for s in range(3):
        b = tuple(abs(x) for x in betas[s]) if absolute else betas[s]
        if has_scattering(k):
            pin, pout = scattering_kernels(k, b)
            pin = pin * cw[:, None]     # [z, i, j, l]
            pout = pout * cw[:, None]
            jac[:, s, 0, 0] = pin[..., 0]
            jac[:, s, 0, 1] = pin[..., 0] + sgn * pout[..., 0]
            jac[:, s, 0, 2] = pin[..., 1]
            jac[:, s, 0, 3] = pin[..., 1] + sgn * pout[..., 1]
        if "pair_a" in k:
            pa = _species(k["pair_a"], b) * cw[:, None]
            pp = _species(k["pair_p"], b) * cw[:, None]
            jac[:, s, 1, 0] = sgn * pp[..., 0]
            jac[:, s, 1, 1] = pa[..., 0] + sgn * pp[..., 0]
            jac[:, s, 1, 2] = sgn * pp[..., 1]
            jac[:, s, 1, 3] = pa[..., 1] + sgn * pp[..., 1]
    return jac


def jacobian(eps, w, T, eta_e, opts=Options(), chunk=32, absolute=False):
    """Jacobian blocks [z, 3, 2, 4, NE, NE] for zone states T[z], eta_e[z] (no f needed).
    ``absolute``: every block entry as its sum of absolute terms, down to the quadrature
    terms (|H| in the kernels), the error scale of one entry."""
    T = np.asarray(T)
    eta_e = np.asarray(eta_e)
    out = []
    for z0 in range(0, T.shape[0], chunk):
        sl = slice(z0, z0 + chunk)
        out.append(jacobian_blocks(zone_kernels(eps, T[sl], eta_e[sl], opts, absolute), w, opts, absolute))
    return np.concatenate(out)


def forward(eps, w, T, eta_e, f, opts=Options(), chunk=32):
    """eta, chi [z, 3, 2, NE] for zone states T[z], eta_e[z] and distributions f[z, 3, 2, NE]."""
    T = np.asarray(T)
    eta_e = np.asarray(eta_e)
    outs_e, outs_c = [], []
    for z0 in range(0, T.shape[0], chunk):
        sl = slice(z0, z0 + chunk)
        k = zone_kernels(eps, T[sl], eta_e[sl], opts)
        e, c = contract(k, w, f[sl], opts)
        outs_e.append(e)
        outs_c.append(c)
    return np.concatenate(outs_e), np.concatenate(outs_c)


def forward_with_scale(eps, w, T, eta_e, f, opts=Options(), chunk=32, quadrature=False):
    """(eta, chi, A_eta, A_chi): outputs plus their sums of absolute terms. With ``quadrature``
    also (Aq_eta, Aq_chi): the same sums with every kernel replaced by its absolute quadrature
    (|H| in the integrand), the scale of the rounding of a quadrature whose angular weight
    changes sign (l = 1); for l = 0 (H >= 0) it equals A."""
    res = [[], [], [], [], [], []]
    for z0 in range(0, len(T), chunk):
        sl = slice(z0, z0 + chunk)
        k = zone_kernels(eps, np.asarray(T)[sl], np.asarray(eta_e)[sl], opts)
        e, c = contract(k, w, f[sl], opts)
        ae, ac = contract_abs(k, w, f[sl], opts)
        vals = [e, c, ae, ac]
        if quadrature:
            kq = zone_kernels(eps, np.asarray(T)[sl], np.asarray(eta_e)[sl], opts, absolute=True)
            vals += list(contract_abs(kq, w, f[sl], opts))
        for lst, v in zip(res, vals):
            lst.append(v)
    return tuple(np.concatenate(r) for r in res if r)
