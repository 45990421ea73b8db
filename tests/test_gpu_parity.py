"""GPU parity of the HIP rates library against the FP64 CPU oracle (needs a gfx950 GPU).

Relative error of an output y against the oracle value y_ref (same rule, same inputs):
  err = |y - y_ref| / max(|y_ref|, 1e-3 A, 1e-290),
A being the sum of the absolute values of the terms that make up y (computed by the
oracle): it keeps outputs that cancel to near zero (eta1, chi1) or underflow from being
compared on rounding noise. Bars: FP64 path 1e-6 (met with ~1e-12), mixed path 1e-4.

Full-size workloads run in one launch over every zone, exactly as the benchmark runs
them, and sampled zones (always including the min-T, max-T and max-eta_e zones) are
compared with the oracle zone by zone.
"""
import sys

import numpy as np
import pytest

from oracle import grad as ograd
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


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def gpu_forward(inp, precision, nquad, rule, processes=3, eta_fp64=30.0):
    grid = vtx.GridHandle(inp.eps, inp.w)
    opts = vtx.make_opts(precision, nquad, rule, processes, eta_fp64=eta_fp64)
    T, E, f = to_dev(inp.T), to_dev(inp.eta_e), to_dev(inp.f)
    eta, chi = vtx.forward(grid, opts, T, E, f)
    torch.cuda.synchronize()
    return eta.cpu().numpy(), chi.cpu().numpy()


def rel_err(y, ref, A):
    den = np.maximum(np.maximum(np.abs(ref), 1e-3 * A), 1e-290)
    return np.abs(y - ref) / den


def oracle_forward(inp, nquad, rule, processes=3):
    opts = orates.Options(nquad=nquad, rule=rule, processes=processes)
    return orates.forward_with_scale(inp.eps, inp.w, inp.T, inp.eta_e, inp.f, opts)


def check_forward(inp, precision, nquad, rule, tol, processes=3, label=""):
    say(f"[gpu] forward {label} precision={precision} nquad={nquad} rule={rule} nz={inp.T.shape[0]} "
        f"ne={inp.eps.shape[0]} processes={processes}")
    e, c = gpu_forward(inp, precision, nquad, rule, processes)
    re, rc, ae, ac = oracle_forward(inp, nquad, rule, processes)
    err_e, err_c = rel_err(e, re, ae), rel_err(c, rc, ac)
    worst = max(err_e.max(), err_c.max())
    say(f"    max rel err eta0 {err_e[:, :, 0].max():.2e} eta1 {err_e[:, :, 1].max():.2e} "
        f"chi0 {err_c[:, :, 0].max():.2e} chi1 {err_c[:, :, 1].max():.2e}")
    assert np.all(np.isfinite(e)) and np.all(np.isfinite(c))
    assert worst <= tol, worst
    return worst


# ---------------------------------------------------------------------------- forward

def test_small_fp64_laguerre_all_zones():
    inp = synth.make_inputs("small")
    check_forward(inp, "fp64", 32, "laguerre", FP64_TOL, label="small")


def test_small_fp64_panel_and_mixed():
    inp = synth.make_inputs("small")
    check_forward(inp, "fp64", 32, "panel", FP64_TOL, label="small/panel")
    check_forward(inp, "mixed", 32, "panel", MIXED_TOL, label="small/panel")


@pytest.mark.parametrize("processes", [1, 2, 4])
def test_single_process(processes):
    inp = synth.make_inputs("medium", nzones=8)
    check_forward(inp, "fp64", 48, "panel", FP64_TOL, processes, label="medium-8")
    check_forward(inp, "mixed", 48, "panel", MIXED_TOL, processes, label="medium-8")


def test_edge_cases():
    # ragged batch, one bin, the 32-bin maximum, node counts 8 and 64, eta_e at 0 and below
    inp = synth.make_inputs("medium", nzones=37)
    check_forward(inp, "fp64", 8, "panel", FP64_TOL, label="ragged-37/n8")
    eps, w = synth.energy_grid(1, 5.0, 9.0)
    T, eta_e, f = synth.draw_zones(5, 1, eps, (1, 20), (-3, 25), (-2, 5), 0.0, 77)
    check_forward(synth.ZoneInputs(eps, w, T, eta_e, f), "fp64", 16, "panel", FP64_TOL, label="ne=1")
    eps, w = synth.energy_grid(32, 1.0, 400.0)
    T, eta_e, f = synth.draw_zones(3, 32, eps, (0.5, 60), (0, 60), (-2, 15), 0.05, 78)
    check_forward(synth.ZoneInputs(eps, w, T, eta_e, f), "fp64", 64, "panel", FP64_TOL, label="ne=32/n64")
    check_forward(synth.ZoneInputs(eps, w, T, eta_e, f), "mixed", 64, "panel", MIXED_TOL, label="ne=32/n64")
    inp = synth.make_inputs("medium", nzones=4)
    inp.eta_e[:] = [0.0, -5.0, 35.0, 60.0]
    inp.T[:] = [0.5, 60.0, 3.0, 1.0]
    check_forward(inp, "fp64", 48, "panel", FP64_TOL, label="extremes")
    check_forward(inp, "mixed", 48, "panel", MIXED_TOL, label="extremes")


def test_empty_batch_and_stream():
    inp = synth.make_inputs("small", nzones=6)
    grid = vtx.GridHandle(inp.eps, inp.w)
    opts = vtx.make_opts("fp64", 32, "laguerre")
    z = torch.zeros(0, dtype=torch.float64, device=DEV)
    e0, c0 = vtx.forward(grid, opts, z, z, torch.zeros((0, 3, 2, inp.eps.shape[0]), dtype=torch.float64,
                                                       device=DEV))
    assert e0.shape[0] == 0
    T, E, f = to_dev(inp.T), to_dev(inp.eta_e), to_dev(inp.f)
    e1, c1 = vtx.forward(grid, opts, T, E, f)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        e2, c2 = vtx.forward(grid, opts, T, E, f)
    s.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(e1, e2) and torch.equal(c1, c2)


def test_deterministic_and_batch_independent():
    inp = synth.make_inputs("medium", nzones=20)
    for prec in ("fp64", "mixed"):
        a = gpu_forward(inp, prec, 48, "panel")
        b = gpu_forward(inp, prec, 48, "panel")
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        one = gpu_forward(synth.subset(inp, [7]), prec, 48, "panel")
        assert np.array_equal(one[0][0], a[0][7]) and np.array_equal(one[1][0], a[1][7])


# ---------------------------------------------------------------------------- backward

def gpu_backward(inp, ge, gc, precision, nquad, rule, eta_fp64=30.0, processes=3):
    grid = vtx.GridHandle(inp.eps, inp.w)
    opts = vtx.make_opts(precision, nquad, rule, processes, eta_fp64=eta_fp64)
    out = vtx.backward(grid, opts, to_dev(inp.T), to_dev(inp.eta_e), to_dev(inp.f), to_dev(ge), to_dev(gc))
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


def grad_err(g, ref):
    """|g - ref| / max(|ref|, 1e-3 mean|ref|) over one field."""
    floor = 1e-3 * np.mean(np.abs(ref)) + 1e-300
    return np.abs(g - ref) / np.maximum(np.abs(ref), floor)


@pytest.mark.parametrize("name,nq,rule,nz", [("small", 32, "laguerre", 6), ("medium", 48, "panel", 6),
                                             ("large", 64, "panel", 4)])
@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
def test_backward_vs_oracle(name, nq, rule, nz, precision, tol):
    inp = synth.make_inputs(name, nzones=nz)
    ge, gc = synth.random_gradients(nz, inp.eps.shape[0], 3)
    say(f"[gpu] backward {name} {precision} nz={nz}")
    gT, gE, gf = gpu_backward(inp, ge, gc, precision, nq, rule)
    rT, rE, rf = ograd.vjp(inp.eps, inp.w, inp.T, inp.eta_e, inp.f, ge, gc, orates.Options(nquad=nq, rule=rule))
    eT, eE, ef = grad_err(gT, rT).max(), grad_err(gE, rE).max(), grad_err(gf, rf).max()
    say(f"    rel err g_T {eT:.2e} g_eta_e {eE:.2e} g_f {ef:.2e}")
    assert max(eT, eE, ef) <= tol


def test_backward_vs_central_differences():
    """FP64 kernels: backward against central differences of the forward kernel itself."""
    inp = synth.make_inputs("medium", nzones=5)
    ge, gc = synth.random_gradients(5, inp.eps.shape[0], 4)
    gT, gE, gf = gpu_backward(inp, ge, gc, "fp64", 48, "panel")

    def L(T, E, f):
        x = synth.ZoneInputs(inp.eps, inp.w, T, E, f)
        e, c = gpu_forward(x, "fp64", 48, "panel")
        return np.sum(ge * e + gc * c, axis=(1, 2, 3))

    h = 1e-6 * inp.T
    fd = (L(inp.T + h, inp.eta_e, inp.f) - L(inp.T - h, inp.eta_e, inp.f)) / (2 * h)
    assert np.all(np.abs(gT - fd) <= 1e-5 * np.abs(gT) + 1e-9 * np.abs(gT).max())
    h = 1e-6 * np.maximum(np.abs(inp.eta_e), 1.0)
    fd = (L(inp.T, inp.eta_e + h, inp.f) - L(inp.T, inp.eta_e - h, inp.f)) / (2 * h)
    assert np.all(np.abs(gE - fd) <= 1e-5 * np.abs(gE) + 1e-9 * np.abs(gE).max())
    for idx in [(0, 0, 2), (1, 1, 9), (2, 0, 20)]:
        fp, fm = inp.f.copy(), inp.f.copy()
        fp[(slice(None),) + idx] += 1e-6
        fm[(slice(None),) + idx] -= 1e-6
        fd = (L(inp.T, inp.eta_e, fp) - L(inp.T, inp.eta_e, fm)) / 2e-6
        g = gf[(slice(None),) + idx]
        assert np.all(np.abs(g - fd) <= 1e-5 * np.abs(g) + 1e-8 * np.abs(gf).max())


def test_autograd_function():
    inp = synth.make_inputs("small", nzones=4)
    grid = vtx.GridHandle(inp.eps, inp.w)
    opts = vtx.make_opts("fp64", 32, "laguerre")
    T = to_dev(inp.T).requires_grad_(True)
    E = to_dev(inp.eta_e).requires_grad_(True)
    f = to_dev(inp.f).requires_grad_(True)
    ge, gc = synth.random_gradients(4, inp.eps.shape[0], 5)
    eta, chi = vtx.rates(T, E, f, grid, opts)
    (eta * to_dev(ge) + chi * to_dev(gc)).sum().backward()
    gT, gE, gf = gpu_backward(inp, ge, gc, "fp64", 32, "laguerre")
    assert np.array_equal(T.grad.cpu().numpy(), gT)
    assert np.array_equal(E.grad.cpu().numpy(), gE)
    assert np.array_equal(f.grad.cpu().numpy(), gf)


def test_autograd_strided_inputs_and_options_copy():
    """Strided (non-contiguous) T, eta_e, f pass forward and backward; changing the options
    object between forward and backward does not change the gradient."""
    inp = synth.make_inputs("small", nzones=4)
    grid = vtx.GridHandle(inp.eps, inp.w)
    opts = vtx.make_opts("fp64", 32, "laguerre")
    big_T = to_dev(np.stack([inp.T, inp.T + 1.0], axis=1))
    big_E = to_dev(np.stack([inp.eta_e, inp.eta_e - 1.0], axis=1))
    big_f = to_dev(np.concatenate([inp.f, inp.f], axis=3))
    Ts, Es, fs = big_T[:, 0], big_E[:, 0], big_f[..., :inp.eps.shape[0]]
    assert not Ts.is_contiguous() and not Es.is_contiguous() and not fs.is_contiguous()
    Ts, Es, fs = (x.detach().requires_grad_(True) for x in (Ts, Es, fs))
    ge, gc = synth.random_gradients(4, inp.eps.shape[0], 5)
    eta, chi = vtx.rates(Ts, Es, fs, grid, opts)
    opts.nquad = 8   # must not reach the backward
    (eta * to_dev(ge) + chi * to_dev(gc)).sum().backward()
    gT, gE, gf = gpu_backward(inp, ge, gc, "fp64", 32, "laguerre")
    assert np.array_equal(Ts.grad.cpu().numpy(), gT)
    assert np.array_equal(Es.grad.cpu().numpy(), gE)
    assert np.array_equal(fs.grad.cpu().numpy(), gf)


def test_nonfinite_input_stays_in_its_zone():
    """NaN or Inf in one zone's T, eta_e or f leaves every other zone's outputs and gradients
    bit for bit as they were (each workgroup reads only its own zone)."""
    inp = synth.make_inputs("medium", nzones=12)
    ge, gc = synth.random_gradients(12, inp.eps.shape[0], 21)
    for prec in ("fp64", "mixed"):
        e0, c0 = gpu_forward(inp, prec, 48, "panel")
        g0 = gpu_backward(inp, ge, gc, prec, 48, "panel")
        for field, z, val in (("T", 3, np.nan), ("eta_e", 5, np.inf), ("eta_e", 7, np.nan), ("f", 9, np.inf),
                              ("T", 11, -np.inf)):
            bad = synth.subset(inp, np.arange(12))
            if field == "f":
                bad.f[z, 1, 0, 4] = val
            else:
                getattr(bad, field)[z] = val
            e, c = gpu_forward(bad, prec, 48, "panel")
            g = gpu_backward(bad, ge, gc, prec, 48, "panel")
            keep = np.arange(12) != z
            assert np.array_equal(e[keep], e0[keep]) and np.array_equal(c[keep], c0[keep]), (prec, field)
            for a, b in zip(g, g0):
                assert np.array_equal(a[keep], b[keep]), (prec, field)
        say(f"[gpu] non-finite inputs ({prec}): other zones unchanged")


def test_workgroup_size_independence():
    """The rate kernels with 8 waves per zone instead of 4 give the same outputs, gradients,
    fused results and Jacobian blocks, bit for bit, in both precisions and every zone class."""
    inp = synth.make_inputs("medium", nzones=10)
    inp.eta_e[:4] = [45.0, -70.0, 12.0, 33.0]
    ge, gc = synth.random_gradients(10, inp.eps.shape[0], 23)
    grid = vtx.GridHandle(inp.eps, inp.w)
    T, E, f, dge, dgc = to_dev(inp.T), to_dev(inp.eta_e), to_dev(inp.f), to_dev(ge), to_dev(gc)

    def run(precision, processes):
        opts = vtx.make_opts(precision, 48, "panel", processes)
        out = list(vtx.forward(grid, opts, T, E, f)) + list(vtx.backward(grid, opts, T, E, f, dge, dgc))
        out += list(vtx.forward_backward(grid, opts, T, E, f, dge, dgc))
        out += list(vtx.jacobian(grid, opts, T, E, f=f))
        torch.cuda.synchronize()
        return [x.cpu().numpy() for x in out]

    try:
        for precision in ("fp64", "mixed"):
            for processes in (3, 7):
                assert vtx.set_workgroup_waves(4) in (4, 8)
                a = run(precision, processes)
                assert vtx.set_workgroup_waves(8) == 4
                b = run(precision, processes)
                for x, y in zip(a, b):
                    assert np.array_equal(x, y), (precision, processes)
        say("[gpu] 4 and 8 waves per zone: identical results")
    finally:
        vtx.set_workgroup_waves(4)


def test_backward_largest_grid():
    """32 bins, the largest grid: 25 task units per zone over the four waves."""
    eps, w = synth.energy_grid(32, 1.0, 400.0)
    T, eta_e, f = synth.draw_zones(2, 32, eps, (2, 30), (0, 20), (-2, 10), 0.05, 79)
    inp = synth.ZoneInputs(eps, w, T, eta_e, f)
    ge, gc = synth.random_gradients(2, 32, 6)
    say("[gpu] backward ne=32")
    gT, gE, gf = gpu_backward(inp, ge, gc, "fp64", 32, "panel")
    rT, rE, rf = ograd.vjp(eps, w, T, eta_e, f, ge, gc, orates.Options(nquad=32, rule="panel"))
    assert max(grad_err(gT, rT).max(), grad_err(gE, rE).max(), grad_err(gf, rf).max()) <= FP64_TOL


def test_mixed_zone_classes():
    """The mixed path splits zones by |eta_e|: FP32 up to the threshold, FP64 above it (the
    threshold capped at 64). Zones above it match the FP64 path bit for bit (forward and
    backward); the others stay within the mixed bars of the oracle. A lower threshold moves
    zones from the first class to the second."""
    inp = synth.make_inputs("medium", nzones=30)
    inp.eta_e[:12] = [-70.0, -45.0, -31.0, 12.0, 25.0, 31.0, 39.0, 55.0, 63.5, 64.5, 90.0, -16.0]
    inp.T[:12] = [0.6, 1.5, 0.8, 3.0, 0.5, 2.0, 1.0, 0.7, 5.0, 0.9, 4.0, 0.55]
    ge, gc = synth.random_gradients(inp.T.shape[0], inp.eps.shape[0], 8)
    re, rc, ae, ac = oracle_forward(inp, 48, "panel")
    rT, rE, rf = ograd.vjp(inp.eps, inp.w, inp.T, inp.eta_e, inp.f, ge, gc, orates.Options(nquad=48, rule="panel"))
    e64, c64 = gpu_forward(inp, "fp64", 48, "panel")
    g64 = gpu_backward(inp, ge, gc, "fp64", 48, "panel")
    for thr in (30.0, 15.0, 100.0):
        high = np.abs(inp.eta_e) > min(thr, 64.0)
        bulk = ~high
        assert high.sum() >= 3 and bulk.sum() >= 5
        say(f"[gpu] mixed classes at threshold {thr}: {int(bulk.sum())} FP32, {int(high.sum())} FP64")
        em, cm = gpu_forward(inp, "mixed", 48, "panel", eta_fp64=thr)
        assert np.array_equal(em[high], e64[high]) and np.array_equal(cm[high], c64[high])
        gm = gpu_backward(inp, ge, gc, "mixed", 48, "panel", eta_fp64=thr)
        for got, ref in zip(gm, g64):
            assert np.array_equal(got[high], ref[high])
        err = max(rel_err(em[bulk], re[bulk], ae[bulk]).max(), rel_err(cm[bulk], rc[bulk], ac[bulk]).max())
        gerr = max(grad_err(gm[0][bulk], rT[bulk]).max(), grad_err(gm[1][bulk], rE[bulk]).max(),
                   grad_err(gm[2][bulk], rf[bulk]).max())
        say(f"    FP32 zones: forward {err:.2e}, backward {gerr:.2e}")
        assert err <= MIXED_TOL and gerr <= MIXED_TOL


def test_class_threshold_boundaries():
    """Zones exactly at the class boundaries: |eta_e| equal to the threshold stays in the FP32
    class and the next double above it goes to FP64; |eta_e| = 64 is FP32 when the threshold
    is 64 or more (the range cap). An FP64-class zone matches the FP64 path bit for bit and an
    FP32-class zone does not (its FP32 quadrature rounds differently), so bit equality tells
    which class ran a zone; every zone stays within the mixed bar of the oracle (floor 1e-2 of
    the outputs' absolute quadrature scale Aq, the mixed path's metric)."""
    above = np.nextafter(30.0, 31.0)
    inp = synth.make_inputs("medium", nzones=8)
    inp.eta_e[:] = [30.0, -30.0, above, -above, 64.0, -64.0, 12.5, 29.0]
    inp.T[:] = [2.0, 1.0, 2.0, 1.0, 1.5, 3.0, 4.0, 0.8]
    re, rc, _, _, qe, qc = orates.forward_with_scale(inp.eps, inp.w, inp.T, inp.eta_e, inp.f,
                                                     orates.Options(nquad=48, rule="panel"), quadrature=True)
    e64, c64 = gpu_forward(inp, "fp64", 48, "panel")
    expect = {30.0: [False, False, True, True, True, True, False, False],
              64.0: [False] * 8, 100.0: [False] * 8}
    for thr, want in expect.items():
        em, cm = gpu_forward(inp, "mixed", 48, "panel", eta_fp64=thr)
        same = [bool(np.array_equal(em[z], e64[z]) and np.array_equal(cm[z], c64[z])) for z in range(8)]
        err = max(rel_err(em, re, 10.0 * qe).max(), rel_err(cm, rc, 10.0 * qc).max())   # floor 1e-2 Aq
        say(f"[gpu] class boundaries at threshold {thr}: FP64 class {same}, max err {err:.2e}")
        assert same == want
        assert err <= MIXED_TOL


def test_zone_class_tiles():
    """The mixed passes give each workgroup the k-th zone of its class in a tile of 64 zones.
    Tiles all of one class, mixed tiles and a ragged last tile: every zone is written once, by its
    own class (outputs prefilled with NaN), FP64-class zones match the FP64 path bit for bit, and
    each FP32-class zone matches the same zone run alone, bit for bit."""
    rng = np.random.default_rng(31)
    inp = synth.make_inputs("medium", nzones=200)
    nz = inp.T.shape[0]
    eta = rng.uniform(0.0, 28.0, nz) * np.where(rng.random(nz) < 0.5, -1.0, 1.0)
    eta[0:64] = rng.uniform(31.0, 60.0, 64)              # tile 0: FP64 class only
    eta[64:128] = rng.uniform(-28.0, 28.0, 64)           # tile 1: FP32 class only
    mix = rng.random(72) < 0.5                           # tile 2 and the ragged tail: mixed
    eta[128:][mix] = rng.uniform(31.0, 60.0, int(mix.sum())) * np.where(rng.random(int(mix.sum())) < 0.5, -1.0, 1.0)
    inp.eta_e[:] = eta
    high = np.abs(eta) > 30.0
    say(f"[gpu] zone-class tiles: {nz} zones, {int(high.sum())} in the FP64 class")
    grid = vtx.GridHandle(inp.eps, inp.w)
    T, E, f = to_dev(inp.T), to_dev(inp.eta_e), to_dev(inp.f)
    out = {}
    for prec in ("mixed", "fp64"):
        opts = vtx.make_opts(prec, 48, "panel", 3, eta_fp64=30.0)
        e = torch.full((nz, 3, 2, inp.eps.shape[0]), float("nan"), dtype=torch.float64, device=DEV)
        c = torch.full_like(e, float("nan"))
        vtx.forward(grid, opts, T, E, f, eta=e, chi=c)
        torch.cuda.synchronize()
        out[prec] = (e.cpu().numpy(), c.cpu().numpy())
    em, cm = out["mixed"]
    assert np.all(np.isfinite(em)) and np.all(np.isfinite(cm))
    assert np.array_equal(em[high], out["fp64"][0][high]) and np.array_equal(cm[high], out["fp64"][1][high])
    low = np.flatnonzero(~high)
    picks = {int(low[0]), int(low[low < 128][-1]), int(low[low >= 128][0]), int(low[low >= 192][-1])}
    for z in sorted(picks):
        one_e, one_c = gpu_forward(synth.subset(inp, [z]), "mixed", 48, "panel")
        assert np.array_equal(one_e[0], em[z]) and np.array_equal(one_c[0], cm[z]), z
    ge, gc = synth.random_gradients(nz, inp.eps.shape[0], 12)
    gm = gpu_backward(inp, ge, gc, "mixed", 48, "panel")
    g64 = gpu_backward(inp, ge, gc, "fp64", 48, "panel")
    for got, ref in zip(gm, g64):
        assert np.all(np.isfinite(got)) and np.array_equal(got[high], ref[high])
    z = int(np.flatnonzero(~high)[-1])
    one = gpu_backward(synth.subset(inp, [z]), ge[z:z + 1], gc[z:z + 1], "mixed", 48, "panel")
    for a, b in zip(one, gm):
        assert np.array_equal(a[0], b[z])


def test_backward_batch_independent():
    """A zone's gradients do not depend on the other zones of the launch (bit for bit)."""
    inp = synth.make_inputs("medium", nzones=9)
    ge, gc = synth.random_gradients(9, inp.eps.shape[0], 10)
    for prec in ("fp64", "mixed"):
        full = gpu_backward(inp, ge, gc, prec, 48, "panel")
        one = gpu_backward(synth.subset(inp, [5]), ge[5:6], gc[5:6], prec, 48, "panel")
        for a, b in zip(full, one):
            assert np.array_equal(a[5:6], b)


# ------------------------------------------------------------------ positron scattering

def test_positron_scattering_forward():
    """All three processes (VTX_NPS added), over eta_e signs and the degenerate end: the
    mirrored zone's task order is nontrivial for eta_e < 0."""
    inp = synth.make_inputs("medium", nzones=10)
    inp.eta_e[:5] = [-12.0, -3.0, 0.0, 45.0, 60.0]
    inp.T[:5] = [2.0, 8.0, 30.0, 1.5, 0.5]
    check_forward(inp, "fp64", 48, "panel", FP64_TOL, processes=7, label="all processes")
    check_forward(inp, "mixed", 48, "panel", MIXED_TOL, processes=7, label="all processes")
    check_forward(inp, "fp64", 48, "panel", FP64_TOL, processes=5, label="both scatterings")
    small = synth.make_inputs("small", nzones=6)
    check_forward(small, "fp64", 32, "laguerre", FP64_TOL, processes=7, label="small/laguerre")


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
def test_positron_scattering_backward(precision, tol):
    inp = synth.make_inputs("medium", nzones=6)
    inp.eta_e[:3] = [-8.0, 0.5, 30.0]
    ge, gc = synth.random_gradients(6, inp.eps.shape[0], 13)
    for proc in (4, 7):
        say(f"[gpu] backward processes={proc} {precision}")
        gT, gE, gf = gpu_backward(inp, ge, gc, precision, 48, "panel", processes=proc)
        rT, rE, rf = ograd.vjp(inp.eps, inp.w, inp.T, inp.eta_e, inp.f, ge, gc,
                               orates.Options(nquad=48, rule="panel", processes=proc))
        eT, eE, ef = grad_err(gT, rT).max(), grad_err(gE, rE).max(), grad_err(gf, rf).max()
        say(f"    rel err g_T {eT:.2e} g_eta_e {eE:.2e} g_f {ef:.2e}")
        assert max(eT, eE, ef) <= tol


def test_positron_scattering_large_sampled():
    """One launch over 307,200 zones of the large workload with all processes, mixed, sampled
    zones against the oracle."""
    wl = synth.WORKLOADS["large"]
    nz = wl.nzones // wl.chunks
    inp = synth.make_inputs("large", nzones=nz)
    grid = vtx.GridHandle(inp.eps, inp.w)
    opts = vtx.make_opts("mixed", wl.nquad, wl.rule, 7)
    say(f"[gpu] all processes, large chunk of {nz} zones")
    eta, chi = vtx.forward(grid, opts, to_dev(inp.T), to_dev(inp.eta_e), to_dev(inp.f))
    torch.cuda.synchronize()
    idx = synth.sample_zones(inp, 12)
    it = torch.from_numpy(idx).to(DEV)
    e, c = eta.index_select(0, it).cpu().numpy(), chi.index_select(0, it).cpu().numpy()
    del eta, chi
    sub = synth.subset(inp, idx)
    re, rc, ae, ac = oracle_forward(sub, wl.nquad, wl.rule, 7)
    err = max(rel_err(e, re, ae).max(), rel_err(c, rc, ac).max())
    say(f"    sampled {len(idx)} zones, max rel err {err:.2e}")
    assert err <= MIXED_TOL


def test_launch_slicing_over_2_22_zones():
    """A call over more than 2^22 zones is issued as slices: zones on both sides of the slice
    boundary and in the last, short slice equal separate launches over them, bit for bit
    (forward and backward, mixed precision)."""
    nz = (1 << 22) + 300
    say(f"[gpu] slicing: {nz} zones")
    inp = synth.make_inputs("large", nzones=nz)
    wl = synth.WORKLOADS["large"]
    grid = vtx.GridHandle(inp.eps, inp.w)
    opts = vtx.make_opts("mixed", wl.nquad, wl.rule)
    T, E, f = to_dev(inp.T), to_dev(inp.eta_e), to_dev(inp.f)
    eta, chi = vtx.forward(grid, opts, T, E, f)
    gen = torch.Generator(device=DEV)
    gen.manual_seed(14)
    ge = torch.randn(f.shape, dtype=torch.float64, device=DEV, generator=gen)
    gc = torch.randn(f.shape, dtype=torch.float64, device=DEV, generator=gen)
    gT, gE, gf = vtx.backward(grid, opts, T, E, f, ge, gc)
    torch.cuda.synchronize()
    idx = np.array([0, (1 << 22) - 2, (1 << 22) - 1, 1 << 22, (1 << 22) + 1, nz - 1])
    it = torch.from_numpy(idx).to(DEV)
    full = [t.index_select(0, it).cpu().numpy() for t in (eta, chi, gT, gE, gf)]
    ges, gcs = ge.index_select(0, it).contiguous(), gc.index_select(0, it).contiguous()
    del eta, chi, gT, gE, gf, T, E, f, ge, gc
    torch.cuda.empty_cache()
    sub = synth.subset(inp, idx)
    Ts, Es, fs = to_dev(sub.T), to_dev(sub.eta_e), to_dev(sub.f)
    e1, c1 = vtx.forward(grid, opts, Ts, Es, fs)
    g1 = vtx.backward(grid, opts, Ts, Es, fs, ges, gcs)
    torch.cuda.synchronize()
    for a, b in zip(full, [t.cpu().numpy() for t in (e1, c1) + tuple(g1)]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("precision,processes", [("fp64", 3), ("mixed", 3), ("mixed", 7), ("fp64", 7)])
def test_forward_backward_fused(precision, processes):
    """vtx_rates_forward_backward: gradients bit for bit those of the backward; eta, chi within
    rounding of the forward (the kernels come from the backward's quadrature loop) and within
    the bars of the oracle."""
    inp = synth.make_inputs("medium", nzones=14)
    inp.eta_e[:3] = [-6.0, 20.0, 66.0]     # the last takes the FP64 pass when mixed
    ge, gc = synth.random_gradients(14, inp.eps.shape[0], 15)
    grid = vtx.GridHandle(inp.eps, inp.w)
    opts = vtx.make_opts(precision, 48, "panel", processes)
    T, E, f, Ge, Gc = (to_dev(a) for a in (inp.T, inp.eta_e, inp.f, ge, gc))
    say(f"[gpu] fused forward+backward {precision} processes={processes}")
    eta, chi, gT, gE, gf = vtx.forward_backward(grid, opts, T, E, f, Ge, Gc)
    e0, c0 = vtx.forward(grid, opts, T, E, f)
    b = vtx.backward(grid, opts, T, E, f, Ge, Gc)
    torch.cuda.synchronize()
    for x, y in zip((gT, gE, gf), b):
        assert torch.equal(x, y)
    re, rc, ae, ac = oracle_forward(inp, 48, "panel", processes)
    e, c = eta.cpu().numpy(), chi.cpu().numpy()
    close = max(rel_err(e, e0.cpu().numpy(), ae).max(), rel_err(c, c0.cpu().numpy(), ac).max())
    err = max(rel_err(e, re, ae).max(), rel_err(c, rc, ac).max())
    say(f"    vs forward {close:.2e}, vs oracle {err:.2e}")
    assert close <= (1e-12 if precision == "fp64" else 1e-5)
    assert err <= (FP64_TOL if precision == "fp64" else MIXED_TOL)


def test_graph_capture_and_replay():
    """Calls allocate nothing, synchronise nothing and record no memset once the tables exist,
    so forward + backward capture into a HIP graph. Every replay, with eager work between
    replays, equals the eager results bit for bit."""
    inp = synth.make_inputs("medium", nzones=40)
    ge, gc = synth.random_gradients(40, inp.eps.shape[0], 16)
    grid = vtx.GridHandle(inp.eps, inp.w)
    for prec in ("mixed", "fp64"):
        opts = vtx.make_opts(prec, 48, "panel")
        T, E, f, Ge, Gc = (to_dev(a) for a in (inp.T, inp.eta_e, inp.f, ge, gc))
        eta0, chi0 = vtx.forward(grid, opts, T, E, f)           # builds the tables, then the eager reference
        b0 = vtx.backward(grid, opts, T, E, f, Ge, Gc)
        torch.cuda.synchronize()
        outs = (torch.empty_like(eta0), torch.empty_like(chi0), torch.empty_like(b0[0]), torch.empty_like(b0[1]),
                torch.empty_like(b0[2]))
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            vtx.forward(grid, opts, T, E, f, outs[0], outs[1], stream=s)
            vtx.backward(grid, opts, T, E, f, Ge, Gc, outs[2], outs[3], outs[4], stream=s)
        torch.cuda.synchronize()
        for rep in range(3):
            for o in outs:
                o.fill_(float("nan"))
            g.replay()
            torch.cuda.synchronize()
            for o, r in zip(outs, (eta0, chi0) + tuple(b0)):
                assert torch.equal(o, r), (prec, rep)
            vtx.forward(grid, opts, T, E, f)                     # eager work between replays
            torch.cuda.synchronize()
        say(f"[gpu] graph capture {prec}: 3 replays equal to eager")


@pytest.mark.parametrize("precision,tol,gtol", [("fp64", FP64_TOL, FP64_TOL), ("mixed", MIXED_TOL, MIXED_TOL)])
def test_largest_grid_all_entry_points(precision, tol, gtol):
    """32 bins, 64 nodes, all three processes (the largest LDS footprint): forward, backward,
    the fused call, the Jacobian with outputs and the task export against the oracle."""
    from oracle import tabulated as otab
    eps, w = synth.energy_grid(32, 1.0, 400.0)
    T, eta_e, f = synth.draw_zones(3, 32, eps, (1.0, 40.0), (-5.0, 50.0), (-2.0, 12.0), 0.05, 83)
    inp = synth.ZoneInputs(eps, w, T, eta_e, f)
    ge, gc = synth.random_gradients(3, 32, 17)
    grid = vtx.GridHandle(eps, w)
    opts = vtx.make_opts(precision, 64, "panel", 7)
    oo = orates.Options(nquad=64, rule="panel", processes=7)
    Td, Ed, fd, Ged, Gcd = (to_dev(a) for a in (T, eta_e, f, ge, gc))
    say(f"[gpu] ne=32 n=64 all processes {precision}")
    e, c = vtx.forward(grid, opts, Td, Ed, fd)
    re, rc, ae, ac = orates.forward_with_scale(eps, w, T, eta_e, f, oo)
    assert max(rel_err(e.cpu().numpy(), re, ae).max(), rel_err(c.cpu().numpy(), rc, ac).max()) <= tol
    gT, gE, gf = vtx.backward(grid, opts, Td, Ed, fd, Ged, Gcd)
    rT, rE, rf = ograd.vjp(eps, w, T, eta_e, f, ge, gc, oo)
    gerr = max(grad_err(gT.cpu().numpy(), rT).max(), grad_err(gE.cpu().numpy(), rE).max(),
               grad_err(gf.cpu().numpy(), rf).max())
    say(f"    backward rel err {gerr:.2e}")
    assert gerr <= gtol
    e2, c2, gT2, gE2, gf2 = vtx.forward_backward(grid, opts, Td, Ed, fd, Ged, Gcd)
    assert torch.equal(gT2, gT) and torch.equal(gE2, gE) and torch.equal(gf2, gf)
    assert max(rel_err(e2.cpu().numpy(), re, ae).max(), rel_err(c2.cpu().numpy(), rc, ac).max()) <= tol
    J, e3, c3 = vtx.jacobian(grid, opts, Td, Ed, f=fd)
    assert torch.equal(e3, e) and torch.equal(c3, c)
    Jr = orates.jacobian(eps, w, T, eta_e, oo)
    Ja = orates.jacobian(eps, w, T, eta_e, oo, absolute=True)
    jerr = (np.abs(J.cpu().numpy() - Jr) / np.maximum(np.maximum(np.abs(Jr), Ja), 1e-290)).max()
    say(f"    jacobian rel err {jerr:.2e}")
    assert jerr <= tol
    q = vtx.tasks(grid, opts, Td, Ed).cpu().numpy()
    qr = otab.pack(orates.task_quadratures(eps, T, eta_e, oo), 32)
    qa = otab.pack(orates.task_quadratures(eps, T, eta_e, oo, absolute=True), 32)
    assert (np.abs(q - qr) / np.maximum(np.maximum(np.abs(qr), qa), 1e-290)).max() <= tol


def test_input_domain_extremes():
    """|eta_e| up to 700 and T from 0.05 to 300 MeV (beyond every workload's range): finite
    outputs and gradients within the bars, both paths."""
    inp = synth.make_inputs("medium", nzones=12)
    inp.eta_e[:] = [-700.0, -200.0, -65.0, 65.0, 200.0, 700.0, 0.0, 30.0, 60.0, -60.0, 10.0, 64.0]
    inp.T[:] = [0.2, 5.0, 100.0, 0.1, 2.0, 0.5, 150.0, 0.05, 0.05, 0.3, 300.0, 0.5]
    ge, gc = synth.random_gradients(12, inp.eps.shape[0], 18)
    re, rc, ae, ac = oracle_forward(inp, 48, "panel")
    rT, rE, rf = ograd.vjp(inp.eps, inp.w, inp.T, inp.eta_e, inp.f, ge, gc, orates.Options(nquad=48, rule="panel"))
    for prec, tol, gtol in (("fp64", FP64_TOL, FP64_TOL), ("mixed", MIXED_TOL, MIXED_TOL)):
        e, c = gpu_forward(inp, prec, 48, "panel")
        gT, gE, gf = gpu_backward(inp, ge, gc, prec, 48, "panel")
        for a in (e, c, gT, gE, gf):
            assert np.all(np.isfinite(a))
        err = max(rel_err(e, re, ae).max(), rel_err(c, rc, ac).max())
        gerr = max(grad_err(gT, rT).max(), grad_err(gE, rE).max(), grad_err(gf, rf).max())
        say(f"[gpu] domain extremes {prec}: forward {err:.2e}, backward {gerr:.2e}")
        assert err <= tol and gerr <= gtol
