"""GPU parity at the workloads' full size, against stored oracle references (needs a gfx950 GPU).

The whole workload runs in the launches the benchmark times (the large one in 8 chunks of
307,200 zones), then the stored FP64 oracle outputs (tests/golden/ref_<workload>.npz, written
by tests/golden/make_reference.py, which calls only oracle/) are compared on their zone
sample: 4,096 zones forward and 512 backward on the large workload, 1,024 and 128 on the
medium one, stratified over (T, eta_e) with the corner eta_e > 30, T < 2 MeV and the extreme
zones always included. Upstream gradients: synth.pooled_gradients (zone z takes row
z mod 4099), gathered on the device.

Gradients: g_T, g_eta_e against max(|g_ref|, 1e-3 mean |g_ref| of the field); g_f of the FP64 path
likewise, g_f of the mixed path against max(|g_ref|, 1e-2 aq_g_f), aq_g_f the sum of the
absolute values of g_f's terms down to the quadrature (the Aq of the gradient).

Errors: forward |y - y_ref| / max(|y_ref|, floor, 1e-290), the floor from an absolute scale of
the output. The FP64 path: floor 1e-3 A, A = the sum of |terms| of y, bar 1e-6. The mixed path:
floor 1e-2 Aq, Aq the same sum with every kernel taken as its absolute quadrature (|H| in the
integrand), bar 1e-4. The floor follows from FP32 rounding: each of a quadrature's n nodes
carries about k = 8 rounded operations (exp2, reciprocal, products, the accumulation), so its
absolute error is about u sqrt(n k) Aq with u = 2^-24, 1.4e-6 Aq at n = 64; a relative error
of 1e-4 is resolvable only down to |y| of about 1e-2 Aq. Outputs below that are the l = 1
moments in which in- and out-scattering or emission and absorption cancel to 1e-3 of their
terms and more (degenerate zones). For l = 0 (H >= 0) Aq = A. The mixed path's errors with
the FP64 path's floor, 1e-3 A, and the share of entries above 1e-4 by it, are printed beside. Backward |g - g_ref| / max(|g_ref|, 1e-3 mean |g_ref| of
the field), bars 1e-6 and 1e-4. The corner stratum and |eta_e| bands are printed on their own.
"""
import functools
import os
import sys

import numpy as np
import pytest

from paper_1404_1719_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1404_1719_amd import vtx  # noqa: E402

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_reference  # noqa: E402

DEV = "cuda:0"
TOL = {"fp64": 1e-6, "mixed": 1e-4}


def say(msg):
    print(msg, flush=True)


@functools.lru_cache(maxsize=1)
def _inputs(name):
    say(f"[gpu] drawing the full {name} workload ({synth.WORKLOADS[name].nzones} zones)")
    return synth.make_inputs(name)


@functools.lru_cache(maxsize=2)
def _ref(name):
    return make_reference.load(name)


def _chunks(nz, n):
    b = np.linspace(0, nz, n + 1).astype(np.int64)
    return [(int(x), int(y)) for x, y in zip(b[:-1], b[1:]) if y > x]


def fwd_err(y, r, a, floor=1e-3):
    return np.abs(y - r) / np.maximum(np.maximum(np.abs(r), floor * a.astype(np.float64)), 1e-290)


MIXED_FLOOR = 1e-2   # x Aq: FP32 rounding of an n = 64 node quadrature, u sqrt(8 n) / 1e-4


def grad_err(g, r):
    return np.abs(g - r) / np.maximum(np.abs(r), 1e-3 * np.mean(np.abs(r)) + 1e-300)


def corner(inp, idx):
    return (inp.eta_e[idx] > 30.0) & (inp.T[idx] < 2.0)


@pytest.mark.parametrize("name", ["large", "medium"])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_forward_full_size_stored_reference(name, precision):
    wl = synth.WORKLOADS[name]
    inp, ref = _inputs(name), _ref(name)
    grid = vtx.GridHandle(inp.eps, inp.w)
    opts = vtx.make_opts(precision, wl.nquad, wl.rule)
    T, E, f = (torch.from_numpy(a).to(DEV) for a in (inp.T, inp.eta_e, inp.f))
    eta, chi = torch.empty_like(f), torch.empty_like(f)
    chunks = _chunks(T.shape[0], wl.chunks)
    say(f"[gpu] {name} {precision} forward: {len(chunks)} launches over {T.shape[0]} zones; "
        f"{ref['idx'].size} stored zones")
    for a, b in chunks:
        vtx.forward(grid, opts, T[a:b], E[a:b], f[a:b], eta[a:b], chi[a:b])
    torch.cuda.synchronize()
    it = torch.from_numpy(ref["idx"]).to(DEV)
    e, c = eta.index_select(0, it).cpu().numpy(), chi.index_select(0, it).cpu().numpy()
    del T, E, f, eta, chi
    torch.cuda.empty_cache()
    assert np.all(np.isfinite(e)) and np.all(np.isfinite(c))
    strict = {"eta0": fwd_err(e[:, :, 0], ref["eta"][:, :, 0], ref["a_eta"][:, :, 0]),
              "eta1": fwd_err(e[:, :, 1], ref["eta"][:, :, 1], ref["a_eta"][:, :, 1]),
              "chi0": fwd_err(c[:, :, 0], ref["chi"][:, :, 0], ref["a_chi"][:, :, 0]),
              "chi1": fwd_err(c[:, :, 1], ref["chi"][:, :, 1], ref["a_chi"][:, :, 1])}
    quad = {"eta0": fwd_err(e[:, :, 0], ref["eta"][:, :, 0], ref["aq_eta"][:, :, 0], MIXED_FLOOR),
            "eta1": fwd_err(e[:, :, 1], ref["eta"][:, :, 1], ref["aq_eta"][:, :, 1], MIXED_FLOOR),
            "chi0": fwd_err(c[:, :, 0], ref["chi"][:, :, 0], ref["aq_chi"][:, :, 0], MIXED_FLOOR),
            "chi1": fwd_err(c[:, :, 1], ref["chi"][:, :, 1], ref["aq_chi"][:, :, 1], MIXED_FLOOR)}
    errs = strict if precision == "fp64" else quad
    cz = corner(inp, ref["idx"])
    say("    max rel err " + " ".join(f"{k} {v.max():.2e}" for k, v in errs.items()) +
        f"; corner ({int(cz.sum())} zones) " + " ".join(f"{k} {v[cz].max(initial=0):.2e}" for k, v in errs.items()))
    if precision == "mixed":
        n_all = sum(v.size for v in strict.values())
        n_over = sum(int((v > 1e-4).sum()) for v in strict.values())
        say("    output-level floor: " + " ".join(f"{k} {v.max():.2e}" for k, v in strict.items()) +
            f"; entries above 1e-4: {n_over} of {n_all} ({n_over / n_all:.1e})")
    a = np.abs(inp.eta_e[ref["idx"]])
    for lo_, hi_ in ((0, 10), (10, 20), (20, 30), (30, 45), (45, 64)):
        sel = (a > lo_) & (a <= hi_)
        worst = max(v[sel].max(initial=0) for v in errs.values())
        tlow = max(v[sel & (inp.T[ref["idx"]] < 2)].max(initial=0) for v in errs.values())
        say(f"    |eta_e| in ({lo_}, {hi_}]: {int(sel.sum())} zones, worst {worst:.2e}, at T < 2 MeV {tlow:.2e}")
    assert max(v.max() for v in errs.values()) <= TOL[precision]


@pytest.mark.parametrize("name", ["large", "medium"])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_backward_full_size_stored_reference(name, precision):
    wl = synth.WORKLOADS[name]
    inp, ref = _inputs(name), _ref(name)
    grid = vtx.GridHandle(inp.eps, inp.w)
    opts = vtx.make_opts(precision, wl.nquad, wl.rule)
    nz = inp.T.shape[0]
    T, E, f = (torch.from_numpy(a).to(DEV) for a in (inp.T, inp.eta_e, inp.f))
    pe, pc = (torch.from_numpy(a).to(DEV) for a in synth.gradient_pool(wl.ne, int(ref["grad_seed"])))
    rows = torch.arange(nz, device=DEV) % pe.shape[0]
    ge, gc = pe.index_select(0, rows), pc.index_select(0, rows)
    del rows
    gT, gE, gf = torch.empty_like(T), torch.empty_like(T), torch.empty_like(f)
    chunks = _chunks(nz, wl.chunks)
    say(f"[gpu] {name} {precision} backward: {len(chunks)} launches; {ref['idx_b'].size} stored zones")
    for a, b in chunks:
        vtx.backward(grid, opts, T[a:b], E[a:b], f[a:b], ge[a:b], gc[a:b], gT[a:b], gE[a:b], gf[a:b])
    torch.cuda.synchronize()
    it = torch.from_numpy(ref["idx_b"]).to(DEV)
    got = [x.index_select(0, it).cpu().numpy() for x in (gT, gE, gf)]
    del T, E, f, ge, gc, gT, gE, gf, pe, pc
    torch.cuda.empty_cache()
    errs = {k: grad_err(g, ref[k]) for k, g in zip(("g_T", "g_eta_e", "g_f"), got)}
    if precision == "mixed":
        # g_f = J^T g sums kernel entries of both signs over the outputs: its FP32 rounding scales
        # with aq_g_f (absolute quadrature terms), as the forward's with Aq; the field-mean floor
        # is printed beside
        say(f"    g_f with the field-mean floor {errs['g_f'].max():.2e}")
        errs["g_f"] = fwd_err(got[2], ref["g_f"], ref["aq_g_f"], MIXED_FLOOR)
    for g in got:
        assert np.all(np.isfinite(g))
    cz = corner(inp, ref["idx_b"])
    say("    max rel err " + " ".join(f"{k} {v.max():.2e}" for k, v in errs.items()) +
        f"; corner ({int(cz.sum())} zones) " + " ".join(f"{k} {v[cz].max(initial=0):.2e}" for k, v in errs.items()))
    assert max(v.max() for v in errs.values()) <= TOL[precision]
