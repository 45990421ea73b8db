"""Python binding of the rates library (ctypes over include/vtx_rates.h).

Argument marshalling only: every step of the computation runs in the HIP kernels of
``lib/libvtxrates.so``. Tensors must be CUDA (HIP) float64 and contiguous; calls are
enqueued on the current torch stream (or the given one) and do not synchronise.
Raises RuntimeError if the library is not built or a call fails -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libvtxrates.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "vtx_rates.h")

VTX_OK, VTX_EINVAL, VTX_EDEVICE, VTX_EHIP, VTX_ENOMEM = 0, 1, 2, 3, 4
VTX_FP64, VTX_MIXED = 0, 1
VTX_RULE_LAGUERRE, VTX_RULE_PANEL = 0, 1
VTX_NES, VTX_PAIR, VTX_NPS = 1, 2, 4


class Grid(ctypes.Structure):
    _fields_ = [("ne", ctypes.c_int32), ("eps", ctypes.POINTER(ctypes.c_double)),
                ("w", ctypes.POINTER(ctypes.c_double))]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("nquad", ctypes.c_int32), ("rule", ctypes.c_int32),
                ("processes", ctypes.c_uint32), ("sin2w", ctypes.c_double), ("eta_fp64", ctypes.c_double)]


class Lattice(ctypes.Structure):
    _fields_ = [("nt", ctypes.c_int32), ("nh", ctypes.c_int32), ("lnT0", ctypes.c_double),
                ("dlnT", ctypes.c_double), ("eta0", ctypes.c_double), ("deta", ctypes.c_double)]


_lib = None


def library():
    """Load (once) and return the ctypes handle; raises if the library was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run python -m paper_1404_1719_amd.build_lib)")
    # torch first: its HIP runtime is the one the device pointers and streams belong to, and the
    # library binds to an already loaded runtime by soname. Loaded first, the library would pull
    # in a second runtime whose devices, pointers and streams are not torch's.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    runtimes = _hip_runtimes()
    if len(runtimes) > 1:
        raise RuntimeError(f"more than one HIP runtime is loaded in this process: {runtimes}")
    vp, i64, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    lib.vtx_opts_default.argtypes = [ctypes.POINTER(Opts)]
    lib.vtx_opts_default.restype = None
    lib.vtx_rates_forward.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Opts), i64, vp, vp, vp, vp, vp, vp]
    lib.vtx_rates_forward.restype = ctypes.c_int
    lib.vtx_rates_forward_mass.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Opts), i64, vp, vp, vp, vp, vp, vp]
    lib.vtx_rates_forward_mass.restype = ctypes.c_int
    lib.vtx_rates_backward.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Opts), i64,
                                       vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.vtx_rates_backward.restype = ctypes.c_int
    lib.vtx_rates_jacobian.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Opts), i64, vp, vp, vp, vp, vp, vp, vp]
    lib.vtx_rates_jacobian.restype = ctypes.c_int
    lib.vtx_rates_forward_backward.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Opts), i64] + [vp] * 11
    lib.vtx_rates_forward_backward.restype = ctypes.c_int
    lib.vtx_task_values.argtypes = [ctypes.c_int32, ctypes.c_uint32]
    lib.vtx_task_values.restype = ctypes.c_int64
    lib.vtx_rates_tasks.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Opts), i64, vp, vp, vp, vp]
    lib.vtx_rates_tasks.restype = ctypes.c_int
    lib.vtx_rates_table_rows.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Opts), i64, vp, vp, vp, vp]
    lib.vtx_rates_table_rows.restype = ctypes.c_int
    lib.vtx_rates_forward_interp.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Opts), ctypes.POINTER(Lattice),
                                             vp, i64, i64, vp, vp, vp, vp, vp, vp]
    lib.vtx_rates_forward_interp.restype = ctypes.c_int
    lib.vtx_ray_system.argtypes = [ctypes.c_int32, i64, ctypes.c_int32, ctypes.c_double] + [vp] * 11
    lib.vtx_ray_system.restype = ctypes.c_int
    lib.vtx_ray_solve.argtypes = [ctypes.c_int32, i64, ctypes.c_int32, vp, vp, vp, vp, vp]
    lib.vtx_ray_solve.restype = ctypes.c_int
    lib.vtx_ray_max_block.argtypes = []
    lib.vtx_ray_max_block.restype = ctypes.c_int
    lib.vtx_strerror.argtypes = [ctypes.c_int]
    lib.vtx_strerror.restype = ctypes.c_char_p
    lib.vtx_abi_version.argtypes = []
    lib.vtx_abi_version.restype = ctypes.c_int
    lib.vtx_set_workgroup_waves.argtypes = [ctypes.c_int]
    lib.vtx_set_workgroup_waves.restype = ctypes.c_int
    lib.vtx_release.argtypes = []
    lib.vtx_release.restype = None
    lib.vtx_gauss_rule.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
    lib.vtx_gauss_rule.restype = ctypes.c_int
    lib.vtx_eval_hpoly.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp]
    lib.vtx_eval_hpoly.restype = ctypes.c_int
    lib.vtx_eval_hmass.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp]
    lib.vtx_eval_hmass.restype = ctypes.c_int
    lib.vtx_task_coefficients.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp]
    lib.vtx_task_coefficients.restype = ctypes.c_int
    _lib = lib
    return lib


def _hip_runtimes():
    """Paths of the HIP runtime libraries mapped into this process."""
    try:
        with open("/proc/self/maps") as fh:
            return sorted({ln.split()[-1] for ln in fh if "libamdhip64" in ln and ln.split()[-1].startswith("/")})
    except OSError:
        return []


def declared_functions():
    """Function names declared in include/vtx_rates.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\**\s+\**(vtx_[a-z_0-9]+)\s*\(", txt, re.M)))


def _check(rc, what):
    if rc != VTX_OK:
        msg = library().vtx_strerror(rc).decode()
        raise RuntimeError(f"{what} failed: {msg} (status {rc})")


class GridHandle:
    """Host copy of an energy grid in the layout the ABI takes (kept alive with the arrays)."""

    def __init__(self, eps, w):
        self.eps = np.ascontiguousarray(eps, dtype=np.float64)
        self.w = np.ascontiguousarray(w, dtype=np.float64)
        if self.eps.shape != self.w.shape or self.eps.ndim != 1:
            raise ValueError("eps and w must be 1-D of equal length")
        self.c = Grid(self.eps.shape[0], self.eps.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                      self.w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))

    @property
    def ne(self):
        return self.eps.shape[0]


def make_opts(precision="fp64", nquad=48, rule="panel", processes=VTX_NES | VTX_PAIR, sin2w=0.2312,
              eta_fp64=30.0):
    o = Opts()
    library().vtx_opts_default(ctypes.byref(o))
    o.precision = {"fp64": VTX_FP64, "mixed": VTX_MIXED}[precision] if isinstance(precision, str) else precision
    o.nquad = nquad
    o.rule = {"laguerre": VTX_RULE_LAGUERRE, "panel": VTX_RULE_PANEL}[rule] if isinstance(rule, str) else rule
    o.processes = processes
    o.sin2w = sin2w
    o.eta_fp64 = eta_fp64
    return o


def _dev_ptr(t, name, shape=None):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def forward(grid: GridHandle, opts: Opts, T, eta_e, f, eta=None, chi=None, stream=None):
    """eta, chi [nz, 3, 2, ne] for T[nz], eta_e[nz], f[nz, 3, 2, ne] (CUDA float64)."""
    import torch
    nz = T.shape[0]
    shp = (nz, 3, 2, grid.ne)
    if eta is None:
        eta = torch.empty(shp, dtype=torch.float64, device=T.device)
    if chi is None:
        chi = torch.empty(shp, dtype=torch.float64, device=T.device)
    rc = library().vtx_rates_forward(ctypes.byref(grid.c), ctypes.byref(opts), nz, _dev_ptr(T, "T", (nz,)),
                                     _dev_ptr(eta_e, "eta_e", (nz,)), _dev_ptr(f, "f", shp),
                                     _dev_ptr(eta, "eta", shp), _dev_ptr(chi, "chi", shp), _stream_handle(stream))
    _check(rc, "vtx_rates_forward")
    return eta, chi


def forward_mass(grid: GridHandle, opts: Opts, T, eta_e, f, eta=None, chi=None, stream=None):
    """eta, chi with the electron mass (vtx_rates_forward_mass; FP64 opts, PANEL rule)."""
    import torch
    nz = T.shape[0]
    shp = (nz, 3, 2, grid.ne)
    if eta is None:
        eta = torch.empty(shp, dtype=torch.float64, device=T.device)
    if chi is None:
        chi = torch.empty(shp, dtype=torch.float64, device=T.device)
    rc = library().vtx_rates_forward_mass(ctypes.byref(grid.c), ctypes.byref(opts), nz, _dev_ptr(T, "T", (nz,)),
                                          _dev_ptr(eta_e, "eta_e", (nz,)), _dev_ptr(f, "f", shp),
                                          _dev_ptr(eta, "eta", shp), _dev_ptr(chi, "chi", shp),
                                          _stream_handle(stream))
    _check(rc, "vtx_rates_forward_mass")
    return eta, chi


def backward(grid: GridHandle, opts: Opts, T, eta_e, f, g_eta, g_chi, g_T=None, g_eta_e=None, g_f=None,
             stream=None):
    """(g_T, g_eta_e, g_f): vector-Jacobian product of (eta, chi) with (g_eta, g_chi)."""
    import torch
    nz = T.shape[0]
    shp = (nz, 3, 2, grid.ne)
    if g_T is None:
        g_T = torch.empty((nz,), dtype=torch.float64, device=T.device)
    if g_eta_e is None:
        g_eta_e = torch.empty((nz,), dtype=torch.float64, device=T.device)
    if g_f is None:
        g_f = torch.empty(shp, dtype=torch.float64, device=T.device)
    rc = library().vtx_rates_backward(
        ctypes.byref(grid.c), ctypes.byref(opts), nz, _dev_ptr(T, "T", (nz,)), _dev_ptr(eta_e, "eta_e", (nz,)),
        _dev_ptr(f, "f", shp), _dev_ptr(g_eta, "g_eta", shp), _dev_ptr(g_chi, "g_chi", shp),
        _dev_ptr(g_T, "g_T", (nz,)), _dev_ptr(g_eta_e, "g_eta_e", (nz,)), _dev_ptr(g_f, "g_f", shp),
        _stream_handle(stream))
    _check(rc, "vtx_rates_backward")
    return g_T, g_eta_e, g_f


def jacobian(grid: GridHandle, opts: Opts, T, eta_e, jac=None, stream=None, f=None):
    """Explicit blocks jac[nz, 3, 2, 4, ne, ne] = d(eta, chi)/df (layout in include/vtx_rates.h).
    With f given, returns (jac, eta, chi) from the same call."""
    import torch
    nz = T.shape[0]
    shp = (nz, 3, 2, 4, grid.ne, grid.ne)
    fs = (nz, 3, 2, grid.ne)
    if jac is None:
        jac = torch.empty(shp, dtype=torch.float64, device=T.device)
    eta = chi = None
    pf = pe = pc = None
    if f is not None:
        eta = torch.empty(fs, dtype=torch.float64, device=T.device)
        chi = torch.empty(fs, dtype=torch.float64, device=T.device)
        pf, pe, pc = _dev_ptr(f, "f", fs), _dev_ptr(eta, "eta", fs), _dev_ptr(chi, "chi", fs)
    rc = library().vtx_rates_jacobian(ctypes.byref(grid.c), ctypes.byref(opts), nz, _dev_ptr(T, "T", (nz,)),
                                      _dev_ptr(eta_e, "eta_e", (nz,)), pf, pe, pc, _dev_ptr(jac, "jac", shp),
                                      _stream_handle(stream))
    _check(rc, "vtx_rates_jacobian")
    return jac if f is None else (jac, eta, chi)


def forward_backward(grid: GridHandle, opts: Opts, T, eta_e, f, g_eta, g_chi, out=None, stream=None):
    """(eta, chi, g_T, g_eta_e, g_f) in one pass (vtx_rates_forward_backward)."""
    import torch
    nz = T.shape[0]
    shp = (nz, 3, 2, grid.ne)
    if out is None:
        out = (torch.empty(shp, dtype=torch.float64, device=T.device),
               torch.empty(shp, dtype=torch.float64, device=T.device),
               torch.empty((nz,), dtype=torch.float64, device=T.device),
               torch.empty((nz,), dtype=torch.float64, device=T.device),
               torch.empty(shp, dtype=torch.float64, device=T.device))
    eta, chi, gT, gE, gf = out
    rc = library().vtx_rates_forward_backward(
        ctypes.byref(grid.c), ctypes.byref(opts), nz, _dev_ptr(T, "T", (nz,)), _dev_ptr(eta_e, "eta_e", (nz,)),
        _dev_ptr(f, "f", shp), _dev_ptr(g_eta, "g_eta", shp), _dev_ptr(g_chi, "g_chi", shp),
        _dev_ptr(eta, "eta", shp), _dev_ptr(chi, "chi", shp), _dev_ptr(gT, "g_T", (nz,)),
        _dev_ptr(gE, "g_eta_e", (nz,)), _dev_ptr(gf, "g_f", shp), _stream_handle(stream))
    _check(rc, "vtx_rates_forward_backward")
    return out


def task_values(ne: int, processes: int) -> int:
    """Doubles per zone of the packed task values."""
    return int(library().vtx_task_values(ne, processes))


def tasks(grid: GridHandle, opts: Opts, T, eta_e, out=None, stream=None, rows=False):
    """Task values [nz, task_values(ne, processes)] (the quadratures before completion); rows:
    in the interpolation variables of a table row (vtx_rates_table_rows)."""
    import torch
    nz = T.shape[0]
    shp = (nz, task_values(grid.ne, opts.processes))
    if out is None:
        out = torch.empty(shp, dtype=torch.float64, device=T.device)
    fn = library().vtx_rates_table_rows if rows else library().vtx_rates_tasks
    rc = fn(ctypes.byref(grid.c), ctypes.byref(opts), nz, _dev_ptr(T, "T", (nz,)), _dev_ptr(eta_e, "eta_e", (nz,)),
            _dev_ptr(out, "tasks", shp), _stream_handle(stream))
    _check(rc, "vtx_rates_table_rows" if rows else "vtx_rates_tasks")
    return out


def lattice_states(lat: Lattice, device):
    """Zone states (T, eta_e) of the lattice nodes, row a nh + b (CUDA float64)."""
    import torch
    a = torch.arange(lat.nt, dtype=torch.float64, device=device).repeat_interleave(lat.nh)
    b = torch.arange(lat.nh, dtype=torch.float64, device=device).repeat(lat.nt)
    return torch.exp(lat.lnT0 + a * lat.dlnT), lat.eta0 + b * lat.deta


def build_table(grid: GridHandle, opts: Opts, lat: Lattice, stream=None):
    """The table of task values over the lattice (vtx_rates_tasks at the lattice states)."""
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    with torch.cuda.stream(s):
        T, E = lattice_states(lat, "cuda")
        return tasks(grid, opts, T.contiguous(), E.contiguous(), stream=s, rows=True)


def forward_interp(grid: GridHandle, opts: Opts, lat: Lattice, table, T, eta_e, f, eta=None, chi=None,
                   stream=None):
    """eta, chi from task values interpolated from the table (vtx_rates_forward_interp)."""
    import torch
    nz = T.shape[0]
    shp = (nz, 3, 2, grid.ne)
    if eta is None:
        eta = torch.empty(shp, dtype=torch.float64, device=T.device)
    if chi is None:
        chi = torch.empty(shp, dtype=torch.float64, device=T.device)
    tshape = (lat.nt * lat.nh, task_values(grid.ne, opts.processes))
    rc = library().vtx_rates_forward_interp(
        ctypes.byref(grid.c), ctypes.byref(opts), ctypes.byref(lat), _dev_ptr(table, "table", tshape),
        tshape[0] * tshape[1], nz,
        _dev_ptr(T, "T", (nz,)), _dev_ptr(eta_e, "eta_e", (nz,)), _dev_ptr(f, "f", shp), _dev_ptr(eta, "eta", shp),
        _dev_ptr(chi, "chi", shp), _stream_handle(stream))
    _check(rc, "vtx_rates_forward_interp")
    return eta, chi


def ray_system(ne, nrays, nzr, dt, jac, f, f_n, f_nm1, eta, chi, lo, up, D=None, rhs=None, stream=None):
    """Diagonal blocks D [nrays*nzr, 6ne, 6ne] and rhs = -G [nrays*nzr, 6ne] of the Newton step
    of the radial sweep (vtx_ray_system; zones laid out ray by ray)."""
    import torch
    nz, nb = nrays * nzr, 6 * ne
    fs = (nz, 3, 2, ne)
    if D is None:
        D = torch.empty((nz, nb, nb), dtype=torch.float64, device=f.device)
    if rhs is None:
        rhs = torch.empty((nz, nb), dtype=torch.float64, device=f.device)
    rc = library().vtx_ray_system(ne, nrays, nzr, float(dt), _dev_ptr(jac, "jac", (nz, 3, 2, 4, ne, ne)),
                                  _dev_ptr(f, "f", fs), _dev_ptr(f_n, "f_n", fs), _dev_ptr(f_nm1, "f_nm1", fs),
                                  _dev_ptr(eta, "eta", fs), _dev_ptr(chi, "chi", fs), _dev_ptr(lo, "lo", (nz, nb)),
                                  _dev_ptr(up, "up", (nz, nb)), _dev_ptr(D, "D", (nz, nb, nb)),
                                  _dev_ptr(rhs, "rhs", (nz, nb)), _stream_handle(stream))
    _check(rc, "vtx_ray_system")
    return D, rhs


def ray_solve(nrays, nzr, lo, D, up, rhs, stream=None):
    """Block-tridiagonal solve along rays, in place (vtx_ray_solve): rhs becomes x, D is
    overwritten. lo, up, rhs [nrays*nzr, nb]; D [nrays*nzr, nb, nb]."""
    nz = nrays * nzr
    nb = rhs.shape[-1]
    rc = library().vtx_ray_solve(nb, nrays, nzr, _dev_ptr(lo, "lo", (nz, nb)), _dev_ptr(D, "D", (nz, nb, nb)),
                                 _dev_ptr(up, "up", (nz, nb)), _dev_ptr(rhs, "rhs", (nz, nb)), _stream_handle(stream))
    _check(rc, "vtx_ray_solve")
    return rhs


def newton_increment(grid: GridHandle, opts: Opts, nrays, nzr, T, eta_e, f, f_n, f_nm1, lo, up, dt, stream=None):
    """Newton increment dF [nrays*nzr, 3, 2, ne] of the radial-sweep system at f: the rates and
    their explicit blocks (one vtx_rates_jacobian call), the system (vtx_ray_system), the solve
    (vtx_ray_solve). Allocates D: 8 (6 ne)^2 bytes per zone."""
    jac, eta, chi = jacobian(grid, opts, T, eta_e, stream=stream, f=f)
    D, rhs = ray_system(grid.ne, nrays, nzr, dt, jac, f, f_n, f_nm1, eta, chi, lo, up, stream=stream)
    del jac
    ray_solve(nrays, nzr, lo, D, up, rhs, stream=stream)
    return rhs.view(f.shape)


def set_workgroup_waves(waves: int) -> int:
    """Diagnostic: run the rate kernels with 4 (default) or 8 waves per zone; returns the previous."""
    prev = library().vtx_set_workgroup_waves(waves)
    if prev < 0:
        raise ValueError("waves must be 4 or 8")
    return prev


def gauss_rule(kind: int, n: int):
    """Host-side Gauss rule of the library: kind 0 Legendre on [0, 1], 1 Laguerre (w e^x)."""
    x = np.zeros(n)
    w = np.zeros(n)
    _check(library().vtx_gauss_rule(kind, n, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "vtx_gauss_rule")
    return x, w


def eval_hpoly(process: int, comp: int, e: float, ep: float, E):
    """Host-side angular weight from the library's coefficient tables."""
    E = np.ascontiguousarray(E, dtype=np.float64)
    out = np.zeros_like(E)
    _check(library().vtx_eval_hpoly(process, comp, e, ep, E.size,
                                    E.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "vtx_eval_hpoly")
    return out



def eval_hmass(process: int, comp: int, e: float, ep: float, E):
    """Host-side angular weight with the electron mass (exact route) from the library's tables."""
    E = np.ascontiguousarray(E, dtype=np.float64)
    out = np.zeros_like(E)
    _check(library().vtx_eval_hmass(process, comp, e, ep, E.size,
                                    E.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "vtx_eval_hmass")
    return out

def task_coefficients(process: int, e: float, ep: float):
    """Host copy of one task's coefficient table (32 / 26 doubles, layout in include/vtx_rates.h)."""
    out = np.zeros(32)
    _check(library().vtx_task_coefficients(process, e, ep, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "vtx_task_coefficients")
    return out if process == VTX_NES else out[:26]


def _make_function():
    import torch

    class VtxRates(torch.autograd.Function):
        """(T, eta_e, f) -> (eta, chi) with the hand-written backward kernel."""

        @staticmethod
        def forward(ctx, T, eta_e, f, grid, opts):
            # the contiguous operands the forward used, and a copy of the options, so that the
            # backward sees exactly the forward's inputs whatever the caller changes later
            Tc, Ec, fc = T.contiguous(), eta_e.contiguous(), f.contiguous()
            ctx.grid = grid
            ctx.opts = Opts.from_buffer_copy(opts)
            ctx.save_for_backward(Tc, Ec, fc)
            return forward(grid, ctx.opts, Tc, Ec, fc)

        @staticmethod
        def backward(ctx, g_eta, g_chi):
            T, eta_e, f = ctx.saved_tensors
            if g_eta is None:
                g_eta = torch.zeros_like(f)
            if g_chi is None:
                g_chi = torch.zeros_like(f)
            gT, gE, gf = backward(ctx.grid, ctx.opts, T, eta_e, f, g_eta.contiguous(), g_chi.contiguous())
            return gT, gE, gf, None, None

    return VtxRates


_fn = None


def rates(T, eta_e, f, grid: GridHandle, opts: Opts):
    """Differentiable (eta, chi) = rates(T, eta_e, f)."""
    global _fn
    if _fn is None:
        _fn = _make_function()
    return _fn.apply(T, eta_e, f, grid, opts)
