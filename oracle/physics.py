"""Physical constants and weak couplings (oracle; test infrastructure only).

The paper gives no interaction physics (its Sect. 2.1 only lists the rates as a model
component). Readings used here:
* 4-fermion V-A interaction, massless e+-; |M|^2 summed over e+- spins is
  32 G_F^2 [beta_I (..)(..) + beta_II (..)(..)] with beta_I = (C_V + C_A)^2,
  beta_II = (C_V - C_A)^2;
* nu_e: C_V = 1/2 + 2 s_W, C_A = +1/2; anti-nu_e: same C_V, C_A = -1/2 (beta_I <-> beta_II);
* nu_x stands for nu_mu, anti-nu_mu, nu_tau, anti-nu_tau: C_V = -1/2 + 2 s_W, C_A = -1/2,
  averaged over particle/antiparticle so beta_I = beta_II = ((C_V+C_A)^2 + (C_V-C_A)^2)/2;
  its pair partner is nu_x itself.
The overall scale beyond G_F (s_W) is a convention: parity unpinned. With the electron mass
(oracle.massive) the matrix element gains m^2 (q.q') beta_III, beta_III = C_V^2 - C_A^2.
"""
import math

G_F = 1.1663787e-11          # MeV^-2
HBARC = 1.973269804e-11      # MeV cm
C0 = 1.0 / (4.0 * math.pi ** 2 * HBARC)   # cm^-1 per (MeV^-2 * MeV^3): the d^3q'/(2 pi)^3 measure
SIN2W = 0.2312
NU_E, NU_EBAR, NU_X = 0, 1, 2
PARTNER = (NU_EBAR, NU_E, NU_X)


def couplings(sin2w: float = SIN2W, electron_mass: bool = False):
    """beta[s] = (beta_I, beta_II) for species s in (nu_e, anti-nu_e, nu_x); with the electron
    mass a third entry beta_III = C_V^2 - C_A^2, the same for a species and its antiparticle
    (C_A -> -C_A), so nu_x's average over both is that of nu_mu."""
    cv_e = 0.5 + 2.0 * sin2w
    b_e = ((cv_e + 0.5) ** 2, (cv_e - 0.5) ** 2)
    cv_x = -0.5 + 2.0 * sin2w
    avg = 0.5 * ((cv_x - 0.5) ** 2 + (cv_x + 0.5) ** 2)
    out = ((b_e[0], b_e[1]), (b_e[1], b_e[0]), (avg, avg))
    if electron_mass:
        m_e, m_x = cv_e * cv_e - 0.25, cv_x * cv_x - 0.25
        out = (out[0] + (m_e,), out[1] + (m_e,), out[2] + (m_x,))
    return out
