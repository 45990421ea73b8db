"""Pins for the oracle's explicit Jacobian blocks (oracle.rates.jacobian).

The blocks are defined as the coefficients of f in the contraction. They are pinned against
two other routes through the oracle that do not use them: the forward contraction itself,
through exact linearity in f (J f = out(f) - out(0)), and the complex-step f-gradient of
oracle.grad (J^T g = dL/df for L = sum g . out)."""
import numpy as np
import pytest

from oracle import grad, physics, rates, rule
from paper_1404_1719_amd import synth

SOURCE = ((0, 1, 2), physics.PARTNER)   # species whose f block p multiplies


def apply_jacobian(jac, f):
    """out[z, s, m, i] for m = 0, 1 of eta and chi from the blocks and f[z, s, m, j]."""
    nz, _, _, ne = f.shape
    eta = np.zeros((nz, 3, 2, ne))
    chi = np.zeros((nz, 3, 2, ne))
    for s in range(3):
        for p in range(2):
            sp = SOURCE[p][s]
            for o in range(4):
                m = o // 2
                v = np.einsum("zij,zj->zi", jac[:, s, p, o], f[:, sp, m])
                (eta if o % 2 == 0 else chi)[:, s, m] += v
    return eta, chi


def transpose_apply(jac, g_eta, g_chi):
    """g_f[z, s', m, j] = sum over blocks of jac^T applied to the upstream gradients."""
    nz, _, _, ne = g_eta.shape
    gf = np.zeros((nz, 3, 2, ne))
    for s in range(3):
        for p in range(2):
            sp = SOURCE[p][s]
            for o in range(4):
                m = o // 2
                g = (g_eta if o % 2 == 0 else g_chi)[:, s, m]
                gf[:, sp, m] += np.einsum("zij,zi->zj", jac[:, s, p, o], g)
    return gf


@pytest.mark.parametrize("workload,nq,rl", [("small", 32, rule.RULE_LAGUERRE), ("medium", 48, rule.RULE_PANEL)])
def test_jacobian_reproduces_contraction(workload, nq, rl):
    inp = synth.make_inputs(workload, nzones=3)
    opts = rates.Options(nquad=nq, rule=rl)
    jac = rates.jacobian(inp.eps, inp.w, inp.T, inp.eta_e, opts)
    ne = inp.eps.shape[0]
    assert jac.shape == (3, 3, 2, 4, ne, ne)
    e1, c1, ae, ac = rates.forward_with_scale(inp.eps, inp.w, inp.T, inp.eta_e, inp.f, opts)
    e0, c0 = rates.forward(inp.eps, inp.w, inp.T, inp.eta_e, np.zeros_like(inp.f), opts)
    je, jc = apply_jacobian(jac, inp.f)
    assert np.all(np.abs(je - (e1 - e0)) <= 1e-12 * (ae + np.abs(e0)))
    assert np.all(np.abs(jc - (c1 - c0)) <= 1e-12 * (ac + np.abs(c0)))


def test_jacobian_transpose_is_f_gradient():
    inp = synth.make_inputs("small", nzones=2)
    opts = rates.Options(nquad=32, rule=rule.RULE_LAGUERRE)
    ge, gc = synth.random_gradients(2, inp.eps.shape[0], 3)
    _, _, gf = grad.vjp(inp.eps, inp.w, inp.T, inp.eta_e, inp.f, ge, gc, opts)
    jac = rates.jacobian(inp.eps, inp.w, inp.T, inp.eta_e, opts)
    got = transpose_apply(jac, ge, gc)
    scale = transpose_apply(rates.jacobian(inp.eps, inp.w, inp.T, inp.eta_e, opts, absolute=True),
                            np.abs(ge), np.abs(gc))
    assert np.all(np.abs(got - gf) <= 1e-12 * scale)


def test_jacobian_process_mask_and_structure():
    inp = synth.make_inputs("medium", nzones=2)
    both = rates.jacobian(inp.eps, inp.w, inp.T, inp.eta_e, rates.Options(nquad=32))
    nes = rates.jacobian(inp.eps, inp.w, inp.T, inp.eta_e, rates.Options(nquad=32, processes=rates.PROC_NES))
    pair = rates.jacobian(inp.eps, inp.w, inp.T, inp.eta_e, rates.Options(nquad=32, processes=rates.PROC_PAIR))
    assert np.all(nes[:, :, 1] == 0) and np.all(pair[:, :, 0] == 0)
    assert np.array_equal(nes[:, :, 0], both[:, :, 0]) and np.array_equal(pair[:, :, 1], both[:, :, 1])
    # in = out on the diagonal: the scattering chi blocks vanish there
    d = np.arange(inp.eps.shape[0])
    assert np.all(both[:, :, 0, 1][..., d, d] == 0) and np.all(both[:, :, 0, 3][..., d, d] == 0)
    # emission by pair production lowers eta0 as the partner fills: eta0 blocks are <= 0
    assert np.all(both[:, :, 1, 0] <= 0)


def test_absolute_scale_bounds_the_blocks():
    """The absolute mode (|H| in the quadratures) bounds every entry, equals it for l = 0
    where the angular weights are nonnegative, and exceeds it for some l = 1 entries."""
    inp = synth.make_inputs("medium", nzones=2)
    opts = rates.Options(nquad=48)
    J = rates.jacobian(inp.eps, inp.w, inp.T, inp.eta_e, opts)
    A = rates.jacobian(inp.eps, inp.w, inp.T, inp.eta_e, opts, absolute=True)
    assert np.all(np.abs(J) <= A * (1 + 1e-13))
    assert np.allclose(np.abs(J[:, :, :, 0]), A[:, :, :, 0], rtol=1e-13, atol=0)
    assert np.any(A[:, :, :, 2] > 1.01 * np.abs(J[:, :, :, 2]))
