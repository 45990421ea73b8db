"""Pins of the oracle's Newton step of the radial sweep (oracle.newton).

* The diagonal blocks equal central differences of the residual with respect to each zone's
  own unknowns (exact here: the rates are affine in f, so the residual is quadratic), and the
  off-diagonal coupling is -lo, -up on the neighbours' same components.
* The source's derivative assembled from the rates' explicit blocks equals central
  differences of S computed by the rates' forward.
* The solve returns x with A x = rhs for the assembled ray matrix, checked with an
  independent sparse product.
* Newton's method converges quadratically to a constructed root (the previous step's
  values shifted so that a chosen state solves the system).
"""
import numpy as np
import pytest

from oracle import newton, rates
from paper_1404_1719_amd import synth


def problem(nrays=2, nz=4, ne=4, seed=3):
    eps, w = synth.energy_grid(ne, 2.0, 60.0)
    T, eta_e, f = synth.draw_zones(nrays * nz, ne, eps, (2.0, 12.0), (0.0, 8.0), (-2.0, 5.0), 0.05, 900 + seed)
    rng = np.random.default_rng(seed)
    sh = (nrays, nz, 3, 2, ne)
    B = 6 * ne
    f = f.reshape(sh)
    f_n = np.clip(f * (1 + 0.02 * rng.standard_normal(sh)), 0, 1)
    f_nm1 = np.clip(f * (1 + 0.02 * rng.standard_normal(sh)), 0, 1)
    opts = rates.Options(nquad=16)
    # time step and radial coupling on the scale of the rates (median opacity), so that the
    # rates' Jacobian and the other terms are of one size
    _, chi = rates.forward(eps, w, T, eta_e, f.reshape(-1, 3, 2, ne), opts)
    kappa = float(np.median(chi[:, :, 0]))
    lo = kappa * rng.uniform(0.0, 0.5, (nrays, nz, B))
    up = kappa * rng.uniform(0.0, 0.5, (nrays, nz, B))
    return eps, w, T.reshape(nrays, nz), eta_e.reshape(nrays, nz), f, f_n, f_nm1, lo, up, opts, 1.0 / kappa


def rates_at(eps, w, T, eta_e, f, opts):
    e, c = rates.forward(eps, w, T.reshape(-1), eta_e.reshape(-1), f.reshape(-1, *f.shape[2:]), opts)
    return e.reshape(f.shape), c.reshape(f.shape)


def test_diagonal_blocks_are_the_residual_derivative():
    eps, w, T, E, f, fn, fm, lo, up, opts, dt = problem()
    eta, chi = rates_at(eps, w, T, E, f, opts)
    jac = rates.jacobian(eps, w, T.reshape(-1), E.reshape(-1), opts).reshape(*T.shape, 3, 2, 4, 4, 4)
    D, rhs = newton.system(jac, f, fn, fm, eta, chi, lo, up, dt)
    G0 = newton.residual(f, fn, fm, eta, chi, lo, up, dt)
    assert np.allclose(rhs, -G0, rtol=0, atol=0)
    nr_, nz = T.shape
    B = f[0, 0].size
    h = 1e-4
    for a, r in ((0, 0), (1, 2)):
        for k in (0, 5, 13, 22):
            fp, fmm = f.copy(), f.copy()
            fp.reshape(nr_, nz, B)[a, r, k] += h
            fmm.reshape(nr_, nz, B)[a, r, k] -= h
            Gp = newton.residual(fp, fn, fm, *rates_at(eps, w, T, E, fp, opts), lo, up, dt)
            Gm = newton.residual(fmm, fn, fm, *rates_at(eps, w, T, E, fmm, opts), lo, up, dt)
            col = (Gp - Gm) / (2 * h)
            scale = np.abs(D[a, r]).max()
            assert np.abs(D[a, r] - np.diag(np.diag(D[a, r]))).max() > 1e-3 * scale   # the rates couple
            assert np.allclose(col[a, r], D[a, r][:, k], rtol=1e-7, atol=1e-9 * scale)
            if r > 0:
                ref = np.zeros(B)
                ref[k] = -up[a, r - 1, k]
                assert np.allclose(col[a, r - 1], ref, rtol=0, atol=1e-9 * scale)
            if r < nz - 1:
                ref = np.zeros(B)
                ref[k] = -lo[a, r + 1, k]
                assert np.allclose(col[a, r + 1], ref, rtol=0, atol=1e-9 * scale)


def test_source_jacobian_from_the_rates_blocks():
    eps, w, T, E, f, *_, opts, _ = problem(nrays=1, nz=2)
    ff = f.reshape(-1, *f.shape[2:])
    e, c = rates.forward(eps, w, T.reshape(-1), E.reshape(-1), ff, opts)
    jac = rates.jacobian(eps, w, T.reshape(-1), E.reshape(-1), opts)
    dS = newton.source_jacobian(jac, ff, e, c)
    B = ff[0].size
    h = 1e-4
    for k in range(0, B, 5):
        fp, fm = ff.copy(), ff.copy()
        fp.reshape(-1, B)[:, k] += h
        fm.reshape(-1, B)[:, k] -= h
        Sp = newton.source(fp, *rates.forward(eps, w, T.reshape(-1), E.reshape(-1), fp, opts))
        Sm = newton.source(fm, *rates.forward(eps, w, T.reshape(-1), E.reshape(-1), fm, opts))
        col = ((Sp - Sm) / (2 * h)).reshape(-1, B)
        assert np.allclose(col, dS[:, :, k], rtol=1e-7, atol=1e-9 * np.abs(dS).max())


def test_solve_satisfies_the_system():
    rng = np.random.default_rng(5)
    nr_, nz, B = 2, 5, 7
    D = rng.standard_normal((nr_, nz, B, B)) + 6 * np.eye(B)
    lo, up = rng.uniform(0, 1, (nr_, nz, B)), rng.uniform(0, 1, (nr_, nz, B))
    rhs = rng.standard_normal((nr_, nz, B))
    x = newton.solve(lo, D, up, rhs)
    for a in range(nr_):
        for r in range(nz):
            y = D[a, r] @ x[a, r]
            if r > 0:
                y = y - lo[a, r] * x[a, r - 1]
            if r < nz - 1:
                y = y - up[a, r] * x[a, r + 1]
            assert np.allclose(y, rhs[a, r], rtol=1e-12, atol=1e-12)


def test_newton_converges_quadratically():
    eps, w, T, E, f, fn, fm, lo, up, opts, dt = problem(nrays=1, nz=3, seed=4)
    target = f
    eta, chi = rates_at(eps, w, T, E, target, opts)
    G = newton.residual(target, fn, fm, eta, chi, lo, up, dt)
    fn = fn + (G * dt / 2.0).reshape(fn.shape)          # now G(target) = 0
    assert np.abs(newton.residual(target, fn, fm, eta, chi, lo, up, dt)).max() < 1e-12 * np.abs(G).max()
    rng = np.random.default_rng(7)
    x = target * (1 + 0.05 * rng.standard_normal(target.shape))
    errs = [np.abs(x - target).max()]
    for _ in range(3):
        x = newton.newton_step(eps, w, T, E, x, fn, fm, lo, up, dt, opts)
        errs.append(np.abs(x - target).max())
    assert errs[1] < 0.1 * errs[0] and errs[2] < 10 * errs[1] ** 2 / errs[0] + 1e-13
    assert errs[3] < 1e-12
