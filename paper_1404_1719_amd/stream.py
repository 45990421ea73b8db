"""Chunked streaming of a workload held in host memory through the GPU (forward + backward).

A one-GPU share of a 3-D model (4096 rays x 600 zones) is processed in chunks of rays. The
workload lives in one pinned host allocation: inputs T, eta_e, f, g_eta, g_chi and outputs
eta, chi, g_T, g_eta_e, g_f, in the library's layouts. Per chunk:

* the inputs go host-to-device by DMA on a copy stream, into one of two device buffer sets
  (chunk c + 1 is copied while chunk c computes; a set is reused once both of its chunk's
  calls have finished);
* the forward and the backward of the chunk read the same inputs and nothing of each other
  (the backward recomputes the kernels), so they run at once on two compute streams;
* both write their outputs straight into the pinned host arrays through the arrays' device
  mapping (hipHostGetDevicePointer): no device-to-host copy kernels compete with the rate
  kernels for compute units, and the forward's PCIe writes spread over the whole chunk.

Three streams at the default priority. Orchestration only: every rate is computed by the
library's kernels (vtx_rates_forward, vtx_rates_backward); no arithmetic happens here.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import vtx

IN = ("T", "eta_e", "f", "g_eta", "g_chi")
OUT = ("eta", "chi", "g_T", "g_eta_e", "g_f")


def _hip():
    paths = vtx._hip_runtimes()
    if not paths:
        raise RuntimeError("HIP runtime not loaded")
    return ctypes.CDLL(paths[0])


class Streamer:
    """Forward + backward of nzones zones held in pinned host memory, in ``chunks`` chunks.

    ``host`` holds the pinned arrays (torch CPU tensors sharing one allocation): fill the
    inputs, call ``step()`` and, after ``synchronize()``, read the outputs."""

    def __init__(self, grid: vtx.GridHandle, opts: vtx.Opts, nzones: int, chunks: int = 8, device="cuda:0"):
        import torch
        self.torch = torch
        self.grid, self.opts = grid, opts
        ne = grid.ne
        self.nzones = int(nzones)
        shapes = {"T": (nzones,), "eta_e": (nzones,), "f": (nzones, 3, 2, ne), "g_eta": (nzones, 3, 2, ne),
                  "g_chi": (nzones, 3, 2, ne), "eta": (nzones, 3, 2, ne), "chi": (nzones, 3, 2, ne),
                  "g_T": (nzones,), "g_eta_e": (nzones,), "g_f": (nzones, 3, 2, ne)}
        total = sum(int(np.prod(s)) for s in shapes.values())
        self.pool = torch.empty(total, dtype=torch.float64, pin_memory=True)   # one pinned allocation
        self.host, off = {}, 0
        for k, s in shapes.items():
            n = int(np.prod(s))
            self.host[k] = self.pool[off:off + n].view(s)
            off += n
        dptr = ctypes.c_void_p()
        rc = _hip().hipHostGetDevicePointer(ctypes.byref(dptr), ctypes.c_void_p(self.pool.data_ptr()), 0)
        if rc != 0 or not dptr.value:
            raise RuntimeError(f"hipHostGetDevicePointer failed ({rc})")
        self.mapped = dptr.value
        b = np.linspace(0, nzones, chunks + 1).astype(np.int64)
        self.chunks = [(int(x), int(y)) for x, y in zip(b[:-1], b[1:]) if y > x]
        n = max((y - x for x, y in self.chunks), default=0)
        dev = torch.device(device)
        self.slots = []
        for _ in range(2):
            d = {k: torch.empty((n,) + shapes[k][1:], dtype=torch.float64, device=dev) for k in IN}
            d["fwd_done"], d["bwd_done"], d["used"] = torch.cuda.Event(), torch.cuda.Event(), False
            self.slots.append(d)
        self.s_fwd = torch.cuda.Stream(device=dev)
        self.s_bwd = torch.cuda.Stream(device=dev)
        self.s_h2d = torch.cuda.Stream(device=dev)
        self.bytes_h2d = sum(self.host[k].numel() for k in IN) * 8
        self.bytes_d2h = sum(self.host[k].numel() for k in OUT) * 8

    def _mapped(self, t):
        """Device address of a slice of the pinned pool."""
        return ctypes.c_void_p(self.mapped + (t.data_ptr() - self.pool.data_ptr()))

    def step(self):
        """Enqueue one forward + backward pass over every chunk (returns without waiting)."""
        torch, H = self.torch, self.host
        lib = vtx.library()
        cur = torch.cuda.current_stream()
        for st in (self.s_h2d, self.s_fwd, self.s_bwd):
            st.wait_stream(cur)
        sf, sb = ctypes.c_void_p(self.s_fwd.cuda_stream), ctypes.c_void_p(self.s_bwd.cuda_stream)
        g, o = ctypes.byref(self.grid.c), ctypes.byref(self.opts)
        for c, (a, b) in enumerate(self.chunks):
            d = self.slots[c % 2]
            n = b - a
            ready = torch.cuda.Event()
            with torch.cuda.stream(self.s_h2d):
                if d["used"]:
                    self.s_h2d.wait_event(d["fwd_done"])
                    self.s_h2d.wait_event(d["bwd_done"])
                for k in IN:
                    d[k][:n].copy_(H[k][a:b], non_blocking=True)
                ready.record(self.s_h2d)
            self.s_fwd.wait_event(ready)
            self.s_bwd.wait_event(ready)
            p = {k: ctypes.c_void_p(d[k].data_ptr()) for k in IN}
            rc = lib.vtx_rates_forward(g, o, n, p["T"], p["eta_e"], p["f"], self._mapped(H["eta"][a:b]),
                                       self._mapped(H["chi"][a:b]), sf)
            vtx._check(rc, "vtx_rates_forward")
            rc = lib.vtx_rates_backward(g, o, n, p["T"], p["eta_e"], p["f"], p["g_eta"], p["g_chi"],
                                        self._mapped(H["g_T"][a:b]), self._mapped(H["g_eta_e"][a:b]),
                                        self._mapped(H["g_f"][a:b]), sb)
            vtx._check(rc, "vtx_rates_backward")
            d["fwd_done"].record(self.s_fwd)
            d["bwd_done"].record(self.s_bwd)
            d["used"] = True
        cur.wait_stream(self.s_fwd)
        cur.wait_stream(self.s_bwd)

    def synchronize(self):
        self.s_fwd.synchronize()
        self.s_bwd.synchronize()
