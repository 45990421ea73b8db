"""Host-side checks of the C-ABI library (no GPU needed, no compute launched).

* every function declared in include/vtx_rates.h is exported;
* argument validation returns VTX_EINVAL before touching any device; a CPU-only machine
  gets VTX_EDEVICE for valid arguments; the HIP fault-injection switch gives VTX_EHIP;
* the library's own Gauss rules (Sturm bisection + Newton) agree with numpy's;
* the library's angular-weight coefficient tables (sympy E-polynomials, generated C)
  agree with the oracle's independent Laurent-antiderivative route.
"""
import ctypes
import os

import numpy as np
import pytest

from oracle.angular import h_nes, h_pair
from paper_1404_1719_amd import synth, vtx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

lib = vtx.library()


def test_exports_every_declared_symbol():
    names = vtx.declared_functions()
    assert {"vtx_rates_forward", "vtx_rates_backward", "vtx_rates_jacobian", "vtx_strerror",
            "vtx_abi_version"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_strings():
    assert lib.vtx_abi_version() == 1
    for c in range(5):
        assert lib.vtx_strerror(c)
    assert lib.vtx_strerror(99) == b"unknown status"


def test_default_options():
    o = vtx.Opts()
    lib.vtx_opts_default(ctypes.byref(o))
    assert (o.precision, o.nquad, o.rule, o.processes) == (0, 48, 1, 3)
    assert o.sin2w == 0.2312 and o.eta_fp64 == 30.0


def _call_fwd(grid, opts, nz, ptr=1):
    p = ctypes.c_void_p(ptr) if ptr else None
    return lib.vtx_rates_forward(ctypes.byref(grid.c) if grid else None, ctypes.byref(opts) if opts else None,
                                 nz, p, p, p, p, p, None)


def _call_bwd(grid, opts, nz, ptr=1):
    p = ctypes.c_void_p(ptr) if ptr else None
    return lib.vtx_rates_backward(ctypes.byref(grid.c), ctypes.byref(opts), nz, p, p, p, p, p, p, p, p, None)


def _call_jac(grid, opts, nz, ptr=1, outs=False):
    p = ctypes.c_void_p(ptr) if ptr else None
    q = p if outs else None
    return lib.vtx_rates_jacobian(ctypes.byref(grid.c), ctypes.byref(opts), nz, p, p, q, q, q, p, None)


def _call_fb(grid, opts, nz, ptr=1):
    p = ctypes.c_void_p(ptr) if ptr else None
    return lib.vtx_rates_forward_backward(ctypes.byref(grid.c), ctypes.byref(opts), nz, *([p] * 11), None)


def test_task_value_counts_match_the_oracle_layout():
    from oracle import rates, tabulated
    for ne in (1, 12, 21, 32):
        for proc in range(1, 8):
            assert lib.vtx_task_values(ne, proc) == tabulated.values_per_zone(ne, rates.Options(processes=proc))
    assert lib.vtx_task_values(0, 3) == 0 and lib.vtx_task_values(21, 8) == 0


def test_invalid_arguments():
    eps, w = synth.energy_grid(21, 2.0, 380.0)
    g = vtx.GridHandle(eps, w)
    o = vtx.make_opts()
    assert _call_fwd(None, o, 4) == vtx.VTX_EINVAL
    assert _call_fwd(g, None, 4) == vtx.VTX_EINVAL
    assert _call_fwd(g, o, -1) == vtx.VTX_EINVAL
    assert _call_fwd(g, o, 4, ptr=0) == vtx.VTX_EINVAL         # null device pointers
    assert _call_bwd(g, o, 4, ptr=0) == vtx.VTX_EINVAL
    assert _call_jac(g, o, 4, ptr=0) == vtx.VTX_EINVAL
    assert _call_jac(g, o, -1) == vtx.VTX_EINVAL
    assert _call_jac(g, o, 0) == vtx.VTX_OK
    p1 = ctypes.c_void_p(1)   # f given without eta, chi
    assert lib.vtx_rates_jacobian(ctypes.byref(g.c), ctypes.byref(o), 4, p1, p1, p1, None, None, p1,
                                  None) == vtx.VTX_EINVAL
    assert _call_fb(g, o, 4, ptr=0) == vtx.VTX_EINVAL
    assert _call_fb(g, o, -1) == vtx.VTX_EINVAL
    assert _call_fb(g, o, 0) == vtx.VTX_OK
    p1 = ctypes.c_void_p(1)
    assert lib.vtx_rates_tasks(ctypes.byref(g.c), ctypes.byref(o), 4, p1, p1, None, None) == vtx.VTX_EINVAL
    assert lib.vtx_rates_tasks(ctypes.byref(g.c), ctypes.byref(o), 0, None, None, None, None) == vtx.VTX_OK
    lat = vtx.Lattice(4, 5, 0.0, 0.1, 0.0, 0.5)
    args = [p1] * 6
    n_ok = 4 * 5 * lib.vtx_task_values(21, 3)
    for bad in (vtx.Lattice(1, 5, 0.0, 0.1, 0.0, 0.5), vtx.Lattice(4, 5, 0.0, 0.0, 0.0, 0.5),
                vtx.Lattice(4, 5, 0.0, 0.1, 0.0, -1.0), vtx.Lattice(4, 5, float("nan"), 0.1, 0.0, 0.5)):
        assert lib.vtx_rates_forward_interp(ctypes.byref(g.c), ctypes.byref(o), ctypes.byref(bad), p1, n_ok, 4,
                                            *args, None) == vtx.VTX_EINVAL
    assert lib.vtx_rates_forward_interp(ctypes.byref(g.c), ctypes.byref(o), None, p1, n_ok, 4, *args,
                                        None) == vtx.VTX_EINVAL
    assert lib.vtx_rates_forward_interp(ctypes.byref(g.c), ctypes.byref(o), ctypes.byref(lat), None, n_ok, 4,
                                        *args, None) == vtx.VTX_EINVAL
    assert lib.vtx_rates_forward_interp(ctypes.byref(g.c), ctypes.byref(o), ctypes.byref(lat),
                                        ctypes.c_void_p(8), n_ok, 4, *args, None) == vtx.VTX_EINVAL  # misaligned
    # a table of another process mask (or length) is refused before any launch
    for n_bad in (n_ok - 2, 4 * 5 * lib.vtx_task_values(21, 7), 0):
        assert lib.vtx_rates_forward_interp(ctypes.byref(g.c), ctypes.byref(o), ctypes.byref(lat), p1, n_bad, 4,
                                            *args, None) == vtx.VTX_EINVAL
    assert lib.vtx_rates_table_rows(ctypes.byref(g.c), ctypes.byref(o), 4, p1, p1, None, None) == vtx.VTX_EINVAL
    for field, bad in [("nquad", 6), ("nquad", 50), ("nquad", 68), ("rule", 2), ("precision", 3),
                       ("processes", 0), ("processes", 8), ("sin2w", float("nan"))]:
        ob = vtx.make_opts()
        setattr(ob, field, bad)
        assert _call_fwd(g, ob, 4) == vtx.VTX_EINVAL, (field, bad)
    assert _call_fwd(vtx.GridHandle(eps[::-1].copy(), w), o, 4) == vtx.VTX_EINVAL       # unsorted
    assert _call_fwd(vtx.GridHandle(eps, -w), o, 4) == vtx.VTX_EINVAL                   # negative volume
    big = np.geomspace(1, 100, 33)
    assert _call_fwd(vtx.GridHandle(big, big), o, 4) == vtx.VTX_EINVAL                  # ne > 32
    assert _call_fwd(g, o, 0) == vtx.VTX_OK                                             # empty batch: no-op


def _gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.mark.skipif(_gpu_available(), reason="checks the no-GPU error path")
def test_no_device_is_reported():
    eps, w = synth.energy_grid(12, 2.0, 300.0)
    assert _call_fwd(vtx.GridHandle(eps, w), vtx.make_opts(), 4) == vtx.VTX_EDEVICE
    assert _call_bwd(vtx.GridHandle(eps, w), vtx.make_opts(), 4) == vtx.VTX_EDEVICE
    assert _call_jac(vtx.GridHandle(eps, w), vtx.make_opts(), 4) == vtx.VTX_EDEVICE
    assert _call_jac(vtx.GridHandle(eps, w), vtx.make_opts(), 4, outs=True) == vtx.VTX_EDEVICE
    assert _call_fb(vtx.GridHandle(eps, w), vtx.make_opts(), 4) == vtx.VTX_EDEVICE


def test_fault_injection_reports_hip_error(monkeypatch):
    monkeypatch.setenv("VTX_FAULT_INJECT_HIP", "1")
    eps, w = synth.energy_grid(12, 2.0, 300.0)
    assert _call_fwd(vtx.GridHandle(eps, w), vtx.make_opts(), 4) == vtx.VTX_EHIP
    with pytest.raises(RuntimeError, match="HIP runtime error"):
        vtx._check(vtx.VTX_EHIP, "x")


@pytest.mark.parametrize("n", [1, 2, 8, 12, 16, 32])
def test_gauss_legendre_matches_numpy(n):
    x, w = vtx.gauss_rule(0, n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(x, 0.5 * (xr + 1), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(w, 0.5 * wr, rtol=1e-12, atol=0)


@pytest.mark.parametrize("n", [2, 8, 12, 16, 32])
def test_gauss_laguerre_matches_numpy(n):
    x, w = vtx.gauss_rule(1, n)
    xr, wr = np.polynomial.laguerre.laggauss(n)
    np.testing.assert_allclose(x, xr, rtol=1e-13, atol=0)
    np.testing.assert_allclose(w, wr * np.exp(xr), rtol=1e-9, atol=0)


def test_gauss_laguerre_64_moments():
    """64-point rule (beyond numpy's accurate range): exact on x^p e^-x, p < 128 (checked to p = 60)."""
    import math
    x, w = vtx.gauss_rule(1, 64)
    for p in range(0, 61, 5):
        assert np.isclose(np.sum(w * np.exp(-x) * x ** p), math.factorial(p), rtol=1e-11, atol=0), p


def test_hpoly_tables_match_oracle():
    rng = np.random.default_rng(5)
    eps, _ = synth.energy_grid(21, 2.0, 380.0)
    for _ in range(60):
        i, j = sorted(rng.integers(0, 21, 2))[::-1]
        e, ep = eps[i], eps[j]
        E = np.concatenate([rng.uniform(0.01, 1.5 * ep, 20), rng.uniform(ep, 4 * e + 50, 20)])
        for comp in range(4):
            S, l = 1 + comp // 2, comp % 2
            ref = h_nes(l, S, e, ep, E)
            got = vtx.eval_hpoly(vtx.VTX_NES, comp, e, ep, E)
            scale = np.abs(h_nes(0, S, e, ep, E)) + 1e-300
            assert np.all(np.abs(got - ref) <= 1e-10 * scale + 1e-12 * np.abs(ref).max()), (e, ep, comp)
        Ep = rng.uniform(0.01, e + ep - 0.01, 40)
        for a, b in ((e, ep), (ep, e)):
            for comp in range(4):
                S, l = 1 + comp // 2, comp % 2
                ref = h_pair(l, S, a, b, Ep)
                got = vtx.eval_hpoly(vtx.VTX_PAIR, comp, a, b, Ep)
                # floor: 1e-12 of the piece's peak, which is of order (a b)^2 / max(a, b)
                scale = np.abs(h_pair(0, S, a, b, Ep)) + 1e-3 * (a * b) ** 2 / max(a, b)
                assert np.all(np.abs(got - ref) <= 1e-9 * scale), (a, b, comp)


def test_one_hip_runtime_whatever_the_import_order():
    """Loading the library before anything imports torch must not pull in a second HIP
    runtime: device pointers and streams come from torch's."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1404_1719_amd import vtx\n"
            "vtx.library()\n"
            "import torch\n"
            "print(len(vtx._hip_runtimes()))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == "1"


def _mass_interval(proc, a, b, E, m):
    """(k0, k1) of the momentum-transfer interval with the electron mass (0, 0 if closed)."""
    with np.errstate(invalid="ignore", divide="ignore"):
        if proc == vtx.VTX_NES:
            Ep = E + a - b
            P, Pp = np.sqrt(np.maximum(E * E - m * m, 0)), np.sqrt(np.maximum(Ep * Ep - m * m, 0))
            return (Pp - P), np.minimum(a + b, P + Pp)
        Eb = a + b - E
        P, Pb = np.sqrt(np.maximum(E * E - m * m, 0)), np.sqrt(np.maximum(Eb * Eb - m * m, 0))
        return np.maximum(abs(a - b), np.abs(P - Pb)), P + Pb


def test_hmass_tables_match_oracle():
    """The generated Laurent coefficients of the electron-mass weights (exact route) against the
    oracle's weights, where the kernels take that route: intervals longer than a quarter of
    their distance from k = 0."""
    from oracle import massive
    rng = np.random.default_rng(6)
    eps, _ = synth.energy_grid(21, 2.0, 380.0)
    eps = np.concatenate([[0.3, 0.6, 1.1], eps])
    m = massive.ME
    n_checked = 0
    for _ in range(80):
        i, j = sorted(rng.integers(0, eps.size, 2))[::-1]
        e, ep = eps[i], eps[j]
        E = m + np.concatenate([rng.uniform(0.0, 2 * ep, 30), rng.uniform(0, 4 * e + 50, 30)])
        for proc, fn in ((vtx.VTX_NES, massive.h_nes), (vtx.VTX_PAIR, massive.h_pair)):
            for a, b in ((e, ep), (ep, e)):
                if proc == vtx.VTX_NES and a < b:
                    continue
                Ev = E if proc == vtx.VTX_NES else np.clip(E, m, a + b - m)
                k0, k1 = _mass_interval(proc, a, b, Ev, m)
                Ev = Ev[(k1 - k0) > 0.25 * k0]
                if Ev.size == 0:
                    continue
                n_checked += Ev.size
                scale = sum(np.abs(fn(0, S, a, b, Ev)) for S in (1, 2, 3)) + 1e-300
                for comp in range(6):
                    S, l = (1 + comp // 2, comp % 2) if comp < 4 else (3, comp - 4)
                    got = vtx.eval_hmass(proc, comp, a, b, Ev)
                    ref = fn(l, S, a, b, Ev)
                    assert np.all(np.abs(got - ref) <= 1e-10 * scale), (proc, a, b, comp)
    assert n_checked > 2000
