"""One Newton step of an implicit radial sweep along a ray (oracle; test infrastructure only).

The paper's radial transport sweep is implicit and ray by ray, with a BDF2 time discretisation,
solved by Newton-Raphson with an explicitly built Jacobian and a direct solution of the
linearised system (Sect. 2.1, radial sweep). The transport terms themselves are out of scope
here; the system below is a minimal stated one that consumes the interaction rates and their
Jacobian blocks.

Unknowns of ray zone r: F_r, the 6 NE values f[species][moment][bin] (the rates' f layout).
Residual of zone r (time in units of length, c = 1; step dt; BDF2 weights 3/2, -2, 1/2):

  G_r = (3/2 F_r - 2 F_r^n + 1/2 F_r^{n-1}) / dt + T_r(F) - S_r(F_r),
  T_r(F)_k = (lo_rk + up_rk) F_rk - lo_rk F_{r-1,k} - up_rk F_{r+1,k}   (F_{-1} = F_N = 0),

with lo, up >= 0 given per zone and component (a three-point radial coupling of each
component: upwind advection, lo = v/dr, up = 0, or diffusion, lo = up = D/dr^2), and the
source of the rates' moments (R9 of the library's definition):

  S0 = eta0 - chi0 f0 - 3 chi1 f1,   S1 = eta1 - chi1 f0 - chi0 f1   (per species and bin).

Jacobian: dG_r/dF_r = (3/(2 dt)) I + diag(lo_r + up_r) - dS_r/dF_r, with
  dS0(i)/df_m(j) = d eta0(i)/df_m(j) - f0(i) d chi0(i)/df_m(j) - 3 f1(i) d chi1(i)/df_m(j)
                   - [same species, i = j] (chi0(i) [m = 0] + 3 chi1(i) [m = 1]),
  dS1(i)/df_m(j) = d eta1(i)/df_m(j) - f0(i) d chi1(i)/df_m(j) - f1(i) d chi0(i)/df_m(j)
                   - [same species, i = j] (chi1(i) [m = 0] + chi0(i) [m = 1]),
the rates' derivatives being the explicit Jacobian blocks (rates.jacobian); dG_r/dF_{r-1} =
-diag(lo_r), dG_r/dF_{r+1} = -diag(up_r). The Newton update solves J dF = -G.

Here the whole ray's matrix is assembled densely and solved with numpy's LU (a library step),
which is the plain definition of the solution the library's block elimination must give.
"""
import numpy as np

from . import rates

BDF2 = (1.5, -2.0, 0.5)
SOURCE = ((0, 1, 2), (1, 0, 2))   # species whose f the scattering (p = 0) / pair (p = 1) block multiplies


def source(f, eta, chi):
    """S [z, 3, 2, ne] of the rates' outputs at f."""
    S = np.empty_like(f)
    S[:, :, 0] = eta[:, :, 0] - chi[:, :, 0] * f[:, :, 0] - 3.0 * chi[:, :, 1] * f[:, :, 1]
    S[:, :, 1] = eta[:, :, 1] - chi[:, :, 1] * f[:, :, 0] - chi[:, :, 0] * f[:, :, 1]
    return S


def source_jacobian(jac, f, eta, chi):
    """dS/dF per zone, [z, B, B] with B = 6 ne in the order (species, moment, bin), from the rates'
    explicit blocks jac [z, 3, 2 process, 4 output, ne, ne] (output order eta0, chi0, eta1, chi1)."""
    nz, _, _, ne = f.shape
    B = 6 * ne
    # d out_o^s(i) / d f_m^{s'}(j), o = eta0, chi0, eta1, chi1 with m = o // 2
    dout = np.zeros((nz, 3, 4, ne, 3, 2, ne))
    for s in range(3):
        for p in range(2):
            sp = SOURCE[p][s]
            for o in range(4):
                dout[:, s, o, :, sp, o // 2, :] += jac[:, s, p, o]
    f0, f1 = f[:, :, 0, :], f[:, :, 1, :]
    dS = np.zeros((nz, 3, 2, ne, 3, 2, ne))
    dS[:, :, 0] = (dout[:, :, 0] - f0[:, :, :, None, None, None] * dout[:, :, 1]
                   - 3.0 * f1[:, :, :, None, None, None] * dout[:, :, 3])
    dS[:, :, 1] = (dout[:, :, 2] - f0[:, :, :, None, None, None] * dout[:, :, 3]
                   - f1[:, :, :, None, None, None] * dout[:, :, 1])
    for s in range(3):
        for i in range(ne):
            dS[:, s, 0, i, s, 0, i] -= chi[:, s, 0, i]
            dS[:, s, 0, i, s, 1, i] -= 3.0 * chi[:, s, 1, i]
            dS[:, s, 1, i, s, 0, i] -= chi[:, s, 1, i]
            dS[:, s, 1, i, s, 1, i] -= chi[:, s, 0, i]
    return dS.reshape(nz, B, B)


def residual(f, f_n, f_nm1, eta, chi, lo, up, dt):
    """G [rays, zones, B] of the system above (f, f_n, f_nm1: [rays, zones, 3, 2, ne]; lo, up:
    [rays, zones, B]; eta, chi at f)."""
    nr_, nz = f.shape[:2]
    B = f[0, 0].size
    F = f.reshape(nr_, nz, B)
    S = source(f.reshape(-1, *f.shape[2:]), eta.reshape(-1, *f.shape[2:]), chi.reshape(-1, *f.shape[2:]))
    G = (BDF2[0] * F + BDF2[1] * f_n.reshape(nr_, nz, B) + BDF2[2] * f_nm1.reshape(nr_, nz, B)) / dt
    G = G + (lo + up) * F
    G[:, 1:] -= lo[:, 1:] * F[:, :-1]
    G[:, :-1] -= up[:, :-1] * F[:, 1:]
    return G - S.reshape(nr_, nz, B)


def system(jac, f, f_n, f_nm1, eta, chi, lo, up, dt):
    """Diagonal blocks D [rays, zones, B, B] = dG_r/dF_r and right-hand side -G."""
    nr_, nz = f.shape[:2]
    B = f[0, 0].size
    dS = source_jacobian(jac.reshape(-1, *jac.shape[2:]), f.reshape(-1, *f.shape[2:]),
                         eta.reshape(-1, *f.shape[2:]), chi.reshape(-1, *f.shape[2:])).reshape(nr_, nz, B, B)
    D = -dS
    idx = np.arange(B)
    D[:, :, idx, idx] += BDF2[0] / dt + lo + up
    return D, -residual(f, f_n, f_nm1, eta, chi, lo, up, dt)


def solve(lo, D, up, rhs):
    """x of  -lo_r x_{r-1} + D_r x_r - up_r x_{r+1} = rhs_r  along each ray: the ray's whole
    matrix assembled densely and solved by LU (numpy)."""
    nr_, nz, B = rhs.shape
    x = np.empty_like(rhs)
    for a in range(nr_):
        A = np.zeros((nz * B, nz * B))
        for r in range(nz):
            A[r * B:(r + 1) * B, r * B:(r + 1) * B] = D[a, r]
            if r > 0:
                A[r * B + np.arange(B), (r - 1) * B + np.arange(B)] = -lo[a, r]
            if r < nz - 1:
                A[r * B + np.arange(B), (r + 1) * B + np.arange(B)] = -up[a, r]
        x[a] = np.linalg.solve(A, rhs[a].reshape(-1)).reshape(nz, B)
    return x


def newton_step(eps, w, T, eta_e, f, f_n, f_nm1, lo, up, dt, opts):
    """One Newton update f + dF along rays: T, eta_e [rays, zones], f... [rays, zones, 3, 2, ne]."""
    nr_, nz = T.shape
    ff = f.reshape(-1, *f.shape[2:])
    eta, chi = rates.forward(eps, w, T.reshape(-1), eta_e.reshape(-1), ff, opts)
    jac = rates.jacobian(eps, w, T.reshape(-1), eta_e.reshape(-1), opts)
    D, rhs = system(jac.reshape(nr_, nz, *jac.shape[1:]), f, f_n, f_nm1, eta.reshape(f.shape), chi.reshape(f.shape),
                    lo, up, dt)
    return f + solve(lo, D, up, rhs).reshape(f.shape)
