"""GPU parity of the explicit Jacobian blocks (vtx_rates_jacobian) against the FP64 oracle.

Entry error: |J - J_ref| / max(|J_ref|, A, 1e-290), A the entry's sum of absolute terms down
to the quadrature terms (|H| for the angular weights; the oracle's absolute mode). A single
l = 1 entry is a quadrature whose angular weight changes sign, so its rounding is set by A,
not by the value; the forward's outputs, sums over j, are judged against 1e-3 of their own
absolute sums instead. Bars as for the forward: FP64 1e-6, mixed 1e-4. The blocks are also
checked against the library's own fused paths: J f equals forward(f) - forward(0), and
J^T g equals the backward's g_f.
"""
import sys

import numpy as np
import pytest

from oracle import rates as orates
from paper_1404_1719_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1404_1719_amd import vtx  # noqa: E402

DEV = "cuda:0"
FP64_TOL = 1e-6
MIXED_TOL = 1e-4
SOURCE = ((0, 1, 2), (1, 0, 2))   # species whose f block p multiplies (scattering, pair partner)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def gpu_jacobian(inp, precision, nquad, rule, processes=3, eta_fp64=30.0):
    grid = vtx.GridHandle(inp.eps, inp.w)
    opts = vtx.make_opts(precision, nquad, rule, processes, eta_fp64=eta_fp64)
    jac = vtx.jacobian(grid, opts, to_dev(inp.T), to_dev(inp.eta_e))
    torch.cuda.synchronize()
    return jac.cpu().numpy()


def jac_err(J, ref, absj):
    return np.abs(J - ref) / np.maximum(np.maximum(np.abs(ref), absj), 1e-290)


def check(inp, precision, nquad, rule, tol, processes=3, label=""):
    say(f"[gpu] jacobian {label} precision={precision} nquad={nquad} rule={rule} nz={inp.T.shape[0]} "
        f"ne={inp.eps.shape[0]} processes={processes}")
    J = gpu_jacobian(inp, precision, nquad, rule, processes)
    opts = orates.Options(nquad=nquad, rule=rule, processes=processes)
    ref = orates.jacobian(inp.eps, inp.w, inp.T, inp.eta_e, opts)
    absj = orates.jacobian(inp.eps, inp.w, inp.T, inp.eta_e, opts, absolute=True)
    assert np.all(np.isfinite(J))
    err = jac_err(J, ref, absj)
    err3 = np.abs(J - ref) / np.maximum(np.maximum(np.abs(ref), 1e-3 * absj), 1e-290)
    plain = np.abs(J - ref) / np.maximum(np.abs(ref), 1e-290)
    big = np.abs(ref) >= 1e-3 * np.sum(absj, axis=-1, keepdims=True)
    say(f"    max rel err {err.max():.2e} (floor A), {err3.max():.2e} (floor 1e-3 A; l = 0 "
        f"{err3[:, :, :, :2].max():.2e}, l = 1 {err3[:, :, :, 2:].max():.2e}); over entries >= 1e-3 of their "
        f"row, plain relative error by (process, output): " +
        " ".join(f"{p}{o}:{plain[:, :, p, o][big[:, :, p, o]].max(initial=0):.1e}" for p in range(2) for o in range(4)))
    assert err.max() <= tol
    # l = 0 entries (no sign change in the angular weight) are held to the forward's floor
    assert err3[:, :, :, :2].max() <= tol
    if tol <= 1e-6:
        assert err3.max() <= tol
    return J


def test_small_all_zones():
    inp = synth.make_inputs("small")
    check(inp, "fp64", 32, "laguerre", FP64_TOL, label="small")
    check(inp, "mixed", 32, "laguerre", MIXED_TOL, label="small")


@pytest.mark.parametrize("processes", [1, 2, 3, 4, 7])
def test_medium_and_process_masks(processes):
    inp = synth.make_inputs("medium", nzones=9)
    J = check(inp, "fp64", 48, "panel", FP64_TOL, processes, label="medium-9")
    if processes == 1:
        assert np.all(J[:, :, 1] == 0)
    if processes == 2:
        assert np.all(J[:, :, 0] == 0)
    if processes == 4:
        assert np.all(J[:, :, 1] == 0) and np.any(J[:, :, 0] != 0)
    check(inp, "mixed", 48, "panel", MIXED_TOL, processes, label="medium-9")


def test_edge_cases():
    eps, w = synth.energy_grid(1, 5.0, 9.0)
    T, eta_e, f = synth.draw_zones(3, 1, eps, (1, 20), (-3, 25), (-2, 5), 0.0, 81)
    check(synth.ZoneInputs(eps, w, T, eta_e, f), "fp64", 16, "panel", FP64_TOL, label="ne=1")
    eps, w = synth.energy_grid(32, 1.0, 400.0)
    T, eta_e, f = synth.draw_zones(3, 32, eps, (0.5, 60), (0, 60), (-2, 15), 0.05, 82)
    check(synth.ZoneInputs(eps, w, T, eta_e, f), "fp64", 64, "panel", FP64_TOL, label="ne=32/n64")
    check(synth.ZoneInputs(eps, w, T, eta_e, f), "mixed", 64, "panel", MIXED_TOL, label="ne=32/n64")
    inp = synth.make_inputs("medium", nzones=5)
    inp.eta_e[:] = [0.0, -5.0, 35.0, 60.0, 70.0]     # the last one takes the FP64 pass when mixed
    inp.T[:] = [0.5, 60.0, 3.0, 1.0, 2.0]
    check(inp, "fp64", 48, "panel", FP64_TOL, label="extremes")
    check(inp, "mixed", 48, "panel", MIXED_TOL, label="extremes")
    grid = vtx.GridHandle(inp.eps, inp.w)
    z = torch.zeros(0, dtype=torch.float64, device=DEV)
    assert vtx.jacobian(grid, vtx.make_opts(), z, z).shape[0] == 0


def _apply(J, f):
    nz, _, _, ne = f.shape
    eta, chi = np.zeros((nz, 3, 2, ne)), np.zeros((nz, 3, 2, ne))
    for s in range(3):
        for p in range(2):
            for o in range(4):
                v = np.einsum("zij,zj->zi", J[:, s, p, o], f[:, SOURCE[p][s], o // 2])
                (eta if o % 2 == 0 else chi)[:, s, o // 2] += v
    return eta, chi


def _apply_t(J, ge, gc):
    gf = np.zeros(ge.shape)
    for s in range(3):
        for p in range(2):
            for o in range(4):
                g = (ge if o % 2 == 0 else gc)[:, s, o // 2]
                gf[:, SOURCE[p][s], o // 2] += np.einsum("zij,zi->zj", J[:, s, p, o], g)
    return gf


@pytest.mark.parametrize("precision,tol_f,tol_g", [("fp64", 1e-12, 1e-10), ("mixed", 1e-12, 1e-4)])
def test_consistent_with_fused_paths(precision, tol_f, tol_g):
    """J f = forward(f) - forward(0) (same task values, FP64 contraction in another order);
    J^T g = backward g_f (task values recomputed by the backward's node loop)."""
    inp = synth.make_inputs("medium", nzones=12)
    grid = vtx.GridHandle(inp.eps, inp.w)
    opts = vtx.make_opts(precision, 48, "panel")
    T, E = to_dev(inp.T), to_dev(inp.eta_e)
    J = vtx.jacobian(grid, opts, T, E).cpu().numpy()
    e1, c1 = [t.cpu().numpy() for t in vtx.forward(grid, opts, T, E, to_dev(inp.f))]
    e0, c0 = [t.cpu().numpy() for t in vtx.forward(grid, opts, T, E, to_dev(np.zeros_like(inp.f)))]
    je, jc = _apply(J, inp.f)
    absj = np.abs(J)
    se, sc = _apply(absj, np.abs(inp.f))
    assert np.all(np.abs(je - (e1 - e0)) <= tol_f * (se + np.abs(e0)))
    assert np.all(np.abs(jc - (c1 - c0)) <= tol_f * (sc + np.abs(c0)))
    ge, gc = synth.random_gradients(12, inp.eps.shape[0], 12)
    _, _, gf = vtx.backward(grid, opts, T, E, to_dev(inp.f), to_dev(ge), to_dev(gc))
    gf = gf.cpu().numpy()
    got = _apply_t(J, ge, gc)
    oabs = orates.jacobian(inp.eps, inp.w, inp.T, inp.eta_e, orates.Options(nquad=48, rule="panel"), absolute=True)
    scale = _apply_t(oabs, np.abs(ge), np.abs(gc))
    err = np.max(np.abs(got - gf) / np.maximum(scale, 1e-300))
    say(f"[gpu] {precision}: J^T g vs backward g_f, max err / scale {err:.2e}")
    assert err <= tol_g


def test_large_chunk_sampled():
    """One launch over 307,200 zones of the large workload (the benchmark's chunk), sampled
    zones (min/max T, max eta_e among them) against the oracle."""
    wl = synth.WORKLOADS["large"]
    nz = wl.nzones // wl.chunks
    say(f"[gpu] jacobian large chunk: {nz} zones, {nz * 192 * wl.ne ** 2 / 1e9:.1f} GB of blocks")
    inp = synth.make_inputs("large", nzones=nz)
    grid = vtx.GridHandle(inp.eps, inp.w)
    opts = vtx.make_opts("mixed", wl.nquad, wl.rule)
    jac = vtx.jacobian(grid, opts, to_dev(inp.T), to_dev(inp.eta_e))
    torch.cuda.synchronize()
    idx = synth.sample_zones(inp, 10)
    J = jac.index_select(0, torch.from_numpy(idx).to(DEV)).cpu().numpy()
    del jac
    torch.cuda.empty_cache()
    sub = synth.subset(inp, idx)
    o = orates.Options(nquad=wl.nquad, rule=wl.rule)
    err = jac_err(J, orates.jacobian(sub.eps, sub.w, sub.T, sub.eta_e, o),
                  orates.jacobian(sub.eps, sub.w, sub.T, sub.eta_e, o, absolute=True)).max()
    say(f"    sampled {len(idx)} zones, max rel err {err:.2e}")
    assert np.all(np.isfinite(J)) and err <= MIXED_TOL


@pytest.mark.parametrize("precision,processes", [("fp64", 3), ("mixed", 3), ("mixed", 7)])
def test_jacobian_with_outputs(precision, processes):
    """The Jacobian call given f also returns eta, chi: equal bit for bit to the forward, and
    the blocks equal to the Jacobian-only call."""
    inp = synth.make_inputs("medium", nzones=11)
    inp.eta_e[:2] = [-4.0, 70.0]          # a mirrored task order; the FP64 pass when mixed
    grid = vtx.GridHandle(inp.eps, inp.w)
    opts = vtx.make_opts(precision, 48, "panel", processes)
    T, E, f = to_dev(inp.T), to_dev(inp.eta_e), to_dev(inp.f)
    J0 = vtx.jacobian(grid, opts, T, E)
    J1, e1, c1 = vtx.jacobian(grid, opts, T, E, f=f)
    e0, c0 = vtx.forward(grid, opts, T, E, f)
    torch.cuda.synchronize()
    assert torch.equal(J0, J1) and torch.equal(e0, e1) and torch.equal(c0, c1)
