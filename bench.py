"""Benchmark: zone x (eps, eps') kernel evaluations per second, forward + backward.

One step = forward (eta, chi) + backward (g_T, g_eta_e, g_f) over every zone of the
workload, inputs resident in HBM, in chunks issued back to back on one compute stream.
Default workload: 4096 rays x 600 zones, NE = 21, 64-node rule, mixed precision, 8 chunks.
Prints ONE JSON line (rank 0). Units: zones * NE^2 per second (each unit covers 3 species,
both processes, l = 0, 1, one forward and one backward evaluation).

Also reported: the same step in plain FP64 (speedup of mixed over FP64), the maximal
relative error per output against the FP64 oracle on sampled zones, a roofline entry for
the dominant kernel (algorithmic FLOPs per launch / measured launch time), the oracle
timed on the host cores on a bounded sample, the same step with the workload held in
pinned host memory and streamed through the GPU chunk by chunk (PCIe transfers included),
and the explicit Jacobian blocks timed over one chunk.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1404_1719_amd import synth  # noqa: E402

# Algorithmic floating-point work per quadrature node (transcendental = 1 op, fma = 2):
#   node coordinate and Fermi-Dirac arguments 4; two exp, two adds, one product, one
#   division and the numerator select-product: 7; weight x blocking 1; each angular-weight
#   component a degree-7 polynomial (Horner, 7 fma = 14) plus its accumulation (2).
#   Scattering nodes carry 4 components, pair nodes 2.  Backward adds, per node, the
#   derivative of the blocking factor along T, eta_e and E (10), node motion (4), the
#   adjoint-weighted polynomial and its derivative (14 + 12) and two accumulations (8).
FLOP_FWD_NES, FLOP_FWD_PAIR = 4 + 7 + 1 + 4 * 16, 4 + 7 + 1 + 2 * 16
FLOP_BWD_EXTRA = 10 + 4 + 26 + 8
PEAK_TFLOPS = {"mixed": 157.3, "fp64": 78.6}   # MI355X vector peaks, FP32 / FP64


def algorithmic_flops_per_zone(ne, nquad, backward):
    ntn, ntp = ne * (ne + 1) // 2, ne * ne
    f_nes = FLOP_FWD_NES + (FLOP_BWD_EXTRA if backward else 0)
    f_pair = FLOP_FWD_PAIR + (FLOP_BWD_EXTRA if backward else 0)
    contraction = 3 * ne * ne * (24 if backward else 20)
    return nquad * (ntn * f_nes + ntp * f_pair) + contraction


def kernel_source_hash():
    h = hashlib.sha256()
    for name in ("vtx_kernels.hip", "vtx_internal.h"):
        with open(os.path.join(ROOT, "paper_1404_1719_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_tag):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary, if it is current."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_tag}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_sha") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def valu_issue_from_profiles(kernel_tag):
    """Measured VALU issue rate (instructions x 4 cycles / SIMD cycles) from a committed
    rocprofv3 SQ-counter summary, if it is current."""
    path = os.path.join(ROOT, "profiles", f"valu_{kernel_tag}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_sha") != kernel_source_hash():
        return None
    return {"valu_issue_frac": rec["valu_issue_frac"], "valu_instr_per_zone": rec["valu_instr_per_zone"]}


def cpu_baseline(wl, budget_s=15.0):
    """Oracle forward + backward on a bounded zone sample, spread over the host cores."""
    from concurrent.futures import ProcessPoolExecutor
    ncores = max(1, min(16, os.cpu_count() or 1))
    # calibrate on one zone, then size the sample to the budget
    t0 = time.perf_counter()
    _oracle_chunk((wl.name, [0]))
    per_zone = time.perf_counter() - t0
    nz = int(max(ncores, min(256, budget_s * ncores / max(per_zone, 1e-3))))
    nz = max(ncores, (nz // ncores) * ncores)
    chunks = [(wl.name, list(range(k, nz, ncores))) for k in range(ncores)]
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=ncores) as ex:
        list(ex.map(_oracle_chunk, chunks))
    dt = time.perf_counter() - t0
    units = nz * wl.ne * wl.ne
    return {"value": units / dt, "unit": "zone*(eps,eps')/s", "cores": ncores, "kind": "oracle",
            "sample": f"{nz} zones of the {wl.name} workload, forward + complex-step backward, "
                      f"{ncores} processes, {dt:.1f} s"}


def _oracle_chunk(arg):
    name, idx = arg
    from oracle import grad as ograd
    from oracle import rates as orates
    wl = synth.WORKLOADS[name]
    inp = synth.subset(synth.make_inputs(name, nzones=max(idx) + 1), idx)
    opts = orates.Options(nquad=wl.nquad, rule=wl.rule)
    orates.forward(inp.eps, inp.w, inp.T, inp.eta_e, inp.f, opts)
    ge, gc = synth.random_gradients(len(idx), wl.ne, 9)
    ograd.vjp(inp.eps, inp.w, inp.T, inp.eta_e, inp.f, ge, gc, opts)
    return len(idx)


def sampled_errors(inp, run, wl, count=6):
    """Max relative error per output on sampled zones vs the FP64 oracle (same rule): the
    forward's four outputs, and the backward's g_T, g_eta_e, g_f against the oracle's
    reverse-mode products for the run's own upstream gradients (floor: 1e-3 x the mean
    magnitude of the field, as g_f = K^T g sums terms of both signs)."""
    import torch
    from oracle import grad as ograd
    from oracle import rates as orates
    idx = synth.sample_zones(inp, count, seed=11)
    it = torch.from_numpy(idx).to(run.eta.device)

    def pick(t):
        return t.index_select(0, it).cpu().numpy()

    e, c, ge, gc = pick(run.eta), pick(run.chi), pick(run.g_eta), pick(run.g_chi)
    gT, gE, gf = pick(run.gT), pick(run.gE), pick(run.gf)
    sub = synth.subset(inp, idx)
    opts = orates.Options(nquad=wl.nquad, rule=wl.rule)
    re, rc, ae, ac = orates.forward_with_scale(sub.eps, sub.w, sub.T, sub.eta_e, sub.f, opts)
    rT, rE, rf = ograd.vjp(sub.eps, sub.w, sub.T, sub.eta_e, sub.f, ge, gc, opts)

    def err(y, r, a):
        return float(np.max(np.abs(y - r) / np.maximum(np.maximum(np.abs(r), 1e-3 * a), 1e-290)))

    def gerr(g, r):
        return float(np.max(np.abs(g - r) / np.maximum(np.abs(r), 1e-3 * np.mean(np.abs(r)) + 1e-300)))

    return {"eta0": err(e[:, :, 0], re[:, :, 0], ae[:, :, 0]), "eta1": err(e[:, :, 1], re[:, :, 1], ae[:, :, 1]),
            "chi0": err(c[:, :, 0], rc[:, :, 0], ac[:, :, 0]), "chi1": err(c[:, :, 1], rc[:, :, 1], ac[:, :, 1]),
            "g_T": gerr(gT, rT), "g_eta_e": gerr(gE, rE), "g_f": gerr(gf, rf), "zones": len(idx)}


class Runner:
    """Device-resident buffers of one workload and the chunked two-stream step."""

    def __init__(self, inp, wl, precision, chunks, processes=3):
        import torch
        from paper_1404_1719_amd import vtx
        self.torch, self.vtx = torch, vtx
        dev = torch.device("cuda:0")
        self.grid = vtx.GridHandle(inp.eps, inp.w)
        self.opts = vtx.make_opts(precision, wl.nquad, wl.rule, processes)
        self.nz, self.ne = inp.T.shape[0], wl.ne
        self.T = torch.from_numpy(inp.T).to(dev)
        self.E = torch.from_numpy(inp.eta_e).to(dev)
        self.f = torch.from_numpy(inp.f).to(dev)
        shp = (self.nz, 3, 2, self.ne)
        g = torch.Generator(device=dev)
        g.manual_seed(synth.SEED_BASE + 3000)
        self.g_eta = torch.randn(shp, dtype=torch.float64, device=dev, generator=g)
        self.g_chi = torch.randn(shp, dtype=torch.float64, device=dev, generator=g)
        self.eta = torch.empty(shp, dtype=torch.float64, device=dev)
        self.chi = torch.empty(shp, dtype=torch.float64, device=dev)
        self.gT = torch.empty((self.nz,), dtype=torch.float64, device=dev)
        self.gE = torch.empty((self.nz,), dtype=torch.float64, device=dev)
        self.gf = torch.empty(shp, dtype=torch.float64, device=dev)
        self.streams = [torch.cuda.Stream(device=dev)]   # default priority
        bounds = np.linspace(0, self.nz, chunks + 1).astype(np.int64)
        self.chunks = [(int(a), int(b)) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]

    def step(self, events=None):
        """One forward + backward pass over all chunks, issued on one compute stream.

        With inputs resident in HBM there are no transfers to hide and every chunk fills the
        chip (hundreds of thousands of workgroups), so chunks run back to back; events
        bracket every launch so that launch durations come from the timed region itself."""
        torch, vtx = self.torch, self.vtx
        s = self.streams[0]
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for a, b in self.chunks:
                ev = None
                if events is not None:
                    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
                    ev[0].record(s)
                vtx.forward(self.grid, self.opts, self.T[a:b], self.E[a:b], self.f[a:b], self.eta[a:b],
                            self.chi[a:b], stream=s)
                if ev is not None:
                    ev[1].record(s)
                vtx.backward(self.grid, self.opts, self.T[a:b], self.E[a:b], self.f[a:b], self.g_eta[a:b],
                             self.g_chi[a:b], self.gT[a:b], self.gE[a:b], self.gf[a:b], stream=s)
                if ev is not None:
                    ev[2].record(s)
                    events.append((b - a, ev))
        torch.cuda.current_stream().wait_stream(s)

    def timed(self, steps, warmup):
        """Seconds per step over `steps` timed steps, and the per-launch event records."""
        torch = self.torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        events = []
        t0 = time.perf_counter()
        for _ in range(steps):
            self.step(events)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / max(steps, 1)
        self.events = events
        return dt

    def fused_step(self):
        """Forward and backward of every chunk in one call each (vtx_rates_forward_backward)."""
        torch, vtx = self.torch, self.vtx
        s = self.streams[0]
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for a, b in self.chunks:
                vtx.forward_backward(self.grid, self.opts, self.T[a:b], self.E[a:b], self.f[a:b], self.g_eta[a:b],
                                     self.g_chi[a:b], out=(self.eta[a:b], self.chi[a:b], self.gT[a:b],
                                                           self.gE[a:b], self.gf[a:b]), stream=s)
        torch.cuda.current_stream().wait_stream(s)

    def timed_fused(self, steps, warmup):
        torch = self.torch
        for _ in range(warmup):
            self.fused_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            self.fused_step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / max(steps, 1)

    def launch_times(self):
        """Average forward / backward launch durations (ms) and zones per launch, from the
        events of the timed region."""
        fwd = [ev[0].elapsed_time(ev[1]) for _, ev in self.events]
        bwd = [ev[1].elapsed_time(ev[2]) for _, ev in self.events]
        zones = [n for n, _ in self.events]
        return float(np.mean(fwd)), float(np.mean(bwd)), float(np.mean(zones))


def hip_runtime():
    """ctypes handle of the HIP runtime this process already uses (torch's), never a second copy."""
    import ctypes
    with open("/proc/self/maps") as fh:
        paths = sorted({ln.split()[-1] for ln in fh if "libamdhip64" in ln and ln.split()[-1].startswith("/")})
    if not paths:
        raise RuntimeError("HIP runtime not loaded")
    return ctypes.CDLL(paths[0])


class Streamer:
    """The workload held in pinned host memory and streamed through the GPU chunk by chunk.
    Inputs go host-to-device on a copy stream (DMA engines) into one of two device buffer
    sets. The forward and the backward of a chunk read the same inputs and nothing of each
    other (the backward recomputes the kernels), so they run on two compute streams at once,
    and both write their outputs directly into the pinned host arrays through the arrays'
    device mapping (hipHostGetDevicePointer): no device-to-host copy kernels compete with the
    rate kernels for compute units, and the forward's output writes spread over the whole
    chunk. Three streams, default priority, one hardware queue each (the null stream holds
    the fourth)."""

    IN = ("T", "E", "f", "g_eta", "g_chi")
    OUT = ("eta", "chi", "gT", "gE", "gf")

    def __init__(self, run):
        import ctypes
        torch = run.torch
        self.torch, self.vtx, self.run = torch, run.vtx, run
        src = {"T": run.T, "E": run.E, "f": run.f, "g_eta": run.g_eta, "g_chi": run.g_chi,
               "eta": run.eta, "chi": run.chi, "gT": run.gT, "gE": run.gE, "gf": run.gf}
        total = sum(t.numel() for t in src.values())
        self.pool = torch.empty(total, dtype=torch.float64, pin_memory=True)   # one pinned allocation
        self.host, off = {}, 0
        for k, t in src.items():
            self.host[k] = self.pool[off:off + t.numel()].view(t.shape)
            off += t.numel()
        for k in self.IN:
            self.host[k].copy_(src[k])
        dptr = ctypes.c_void_p()
        rc = hip_runtime().hipHostGetDevicePointer(ctypes.byref(dptr), ctypes.c_void_p(self.pool.data_ptr()), 0)
        if rc != 0 or not dptr.value:
            raise RuntimeError(f"hipHostGetDevicePointer failed ({rc})")
        self.mapped = dptr.value
        self.bytes_in = sum(self.host[k].numel() for k in self.IN) * 8
        self.bytes_out = sum(self.host[k].numel() for k in self.OUT) * 8
        n = max(b - a for a, b in run.chunks)
        dev = run.T.device
        self.slots = []
        for _ in range(2):
            d = {k: torch.empty((n,) + tuple(src[k].shape[1:]), dtype=torch.float64, device=dev) for k in self.IN}
            d["fwd_done"] = torch.cuda.Event()
            d["bwd_done"] = torch.cuda.Event()
            d["used"] = False
            self.slots.append(d)
        self.cf = run.streams[0]
        self.cb = torch.cuda.Stream(device=dev)
        self.h2d = torch.cuda.Stream(device=dev)

    def out_ptr(self, t):
        """Device address of a slice of the pinned host pool."""
        import ctypes
        return ctypes.c_void_p(self.mapped + (t.data_ptr() - self.pool.data_ptr()))

    def step(self):
        import ctypes
        torch, run, H = self.torch, self.run, self.host
        lib = self.vtx.library()
        cur = torch.cuda.current_stream()
        for st in (self.h2d, self.cf, self.cb):
            st.wait_stream(cur)
        sf, sb = ctypes.c_void_p(self.cf.cuda_stream), ctypes.c_void_p(self.cb.cuda_stream)
        g, o = ctypes.byref(run.grid.c), ctypes.byref(run.opts)
        for c, (a, b) in enumerate(run.chunks):
            d = self.slots[c % 2]
            n = b - a
            ready = torch.cuda.Event()
            with torch.cuda.stream(self.h2d):
                if d["used"]:
                    self.h2d.wait_event(d["fwd_done"])
                    self.h2d.wait_event(d["bwd_done"])
                for k in self.IN:
                    d[k][:n].copy_(H[k][a:b], non_blocking=True)
                ready.record(self.h2d)
            self.cf.wait_event(ready)
            self.cb.wait_event(ready)
            p = {k: ctypes.c_void_p(d[k].data_ptr()) for k in self.IN}
            rc = lib.vtx_rates_forward(g, o, n, p["T"], p["E"], p["f"], self.out_ptr(H["eta"][a:b]),
                                       self.out_ptr(H["chi"][a:b]), sf)
            rc = rc or lib.vtx_rates_backward(g, o, n, p["T"], p["E"], p["f"], p["g_eta"], p["g_chi"],
                                              self.out_ptr(H["gT"][a:b]), self.out_ptr(H["gE"][a:b]),
                                              self.out_ptr(H["gf"][a:b]), sb)
            if rc:
                raise RuntimeError(f"rates call failed ({rc})")
            d["fwd_done"].record(self.cf)
            d["bwd_done"].record(self.cb)
            d["used"] = True
        cur.wait_stream(self.cf)
        cur.wait_stream(self.cb)

    def timed(self, steps, warmup):
        torch = self.torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            self.step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / max(steps, 1)


def streaming_leg(run, units, steps, warmup):
    """Whole-job rate with the workload in pinned host memory (PCIe transfers included)."""
    torch = run.torch
    st = Streamer(run)
    t = st.timed(steps, warmup)
    same = bool(torch.equal(st.host["gT"].to(run.gT.device), run.gT) and
                torch.equal(st.host["gf"].to(run.gf.device), run.gf) and
                torch.equal(st.host["eta"].to(run.eta.device), run.eta) and
                torch.equal(st.host["chi"].to(run.chi.device), run.chi))
    out = {"value": units / t, "unit": "zone*(eps,eps')/s", "ms_per_step": t * 1e3, "steps": steps,
           "bytes_h2d": st.bytes_in, "bytes_to_host": st.bytes_out,
           "pcie_GBps": (st.bytes_in + st.bytes_out) / t / 1e9,
           "outputs_equal_resident_run": same,
           "note": "pinned host arrays; inputs by DMA copies into 2 device buffer sets; forward and "
                   "backward of a chunk on two compute streams at once; outputs written by the kernels "
                   "into the mapped host arrays"}
    del st
    torch.cuda.empty_cache()
    return out


def jacobian_leg(inp, wl, precision, launches):
    """Explicit Jacobian blocks over one chunk: launch time (HIP events on the launch stream)
    and the HBM write rate of its 24 NE^2 doubles per zone."""
    import torch
    from paper_1404_1719_amd import vtx
    nz = wl.nzones // wl.chunks
    dev = torch.device("cuda:0")
    grid = vtx.GridHandle(inp.eps, inp.w)
    opts = vtx.make_opts(precision, wl.nquad, wl.rule)
    T = torch.from_numpy(inp.T[:nz]).to(dev)
    E = torch.from_numpy(inp.eta_e[:nz]).to(dev)
    jac = torch.empty((nz, 3, 2, 4, wl.ne, wl.ne), dtype=torch.float64, device=dev)
    s = torch.cuda.Stream(device=dev)
    s.wait_stream(torch.cuda.current_stream())
    ms = []
    with torch.cuda.stream(s):
        vtx.jacobian(grid, opts, T, E, jac, stream=s)
        for _ in range(launches):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record(s)
            vtx.jacobian(grid, opts, T, E, jac, stream=s)
            ev[1].record(s)
            ms.append(ev)
    s.synchronize()
    t = float(np.mean([a.elapsed_time(b) for a, b in ms]))
    written = jac.numel() * 8
    del jac
    torch.cuda.empty_cache()
    tag = f"rates_jacobian_{precision}_{wl.name}"
    return {"zones_per_launch": nz, "launch_ms": t, "bytes_written": written,
            "write_GBps": written / (t * 1e-3) / 1e9, "hbm_peak_GBps": 8000.0,
            "hbm_frac": written / (t * 1e-3) / 8e12, "traffic": traffic_from_profiles(tag), "kernel": tag}


def tabulated_leg(inp, wl, precision, launches, t_direct_ms):
    """Tabulated comparison point: task values on a (ln T, eta_e) lattice over the workload's
    range (built by the library), interpolated per zone over one chunk, against the direct
    forward. Errors: against the FP64 oracle's direct rates on sampled zones, with the A10
    floor of the direct path; and over every zone of the chunk for the l = 0 outputs (which do
    not cancel), against the library's direct forward, |y_tab - y| / max(|y|, 1e-3 max over the
    bins of the same output)."""
    import math
    import torch
    from paper_1404_1719_amd import vtx
    nz = wl.nzones // wl.chunks
    dev = torch.device("cuda:0")
    grid = vtx.GridHandle(inp.eps, inp.w)
    opts = vtx.make_opts(precision, wl.nquad, wl.rule)
    tmin, tmax = float(inp.T.min()), float(inp.T.max())
    emin, emax = float(inp.eta_e.min()), float(inp.eta_e.max())
    dlnT, deta = 0.1, 0.25
    nt = int(math.ceil((math.log(tmax) - math.log(tmin)) / dlnT)) + 1
    nh = int(math.ceil((emax - emin) / deta)) + 1
    lat = vtx.Lattice(nt, nh, math.log(tmin), dlnT, emin, deta)
    s = torch.cuda.Stream(device=dev)
    s.wait_stream(torch.cuda.current_stream())
    T = torch.from_numpy(inp.T[:nz]).to(dev)
    E = torch.from_numpy(inp.eta_e[:nz]).to(dev)
    f = torch.from_numpy(inp.f[:nz]).to(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    with torch.cuda.stream(s):
        table = vtx.build_table(grid, opts, lat, stream=s)   # first build loads its kernel
        ev[0].record(s)
        vtx.build_table(grid, opts, lat, stream=s)
        ev[1].record(s)
        eta, chi = vtx.forward_interp(grid, opts, lat, table, T, E, f, stream=s)
        ms = []
        for _ in range(launches):
            e2 = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            e2[0].record(s)
            vtx.forward_interp(grid, opts, lat, table, T, E, f, eta, chi, stream=s)
            e2[1].record(s)
            ms.append(e2)
        e0, c0 = vtx.forward(grid, opts, T, E, f, stream=s)
    s.synchronize()
    t = float(np.mean([a.elapsed_time(b) for a, b in ms]))

    def err(y, r):
        y, r = y[:, :, 0], r[:, :, 0]
        d = (y - r).abs() / torch.maximum(r.abs(), 1e-3 * r.abs().amax(dim=-1, keepdim=True))
        return {"max": d.max().item(), "median": d.median().item()}

    from oracle import rates as orates
    sub_idx = synth.sample_zones(synth.subset(inp, np.arange(nz)), 6, seed=12)
    it = torch.from_numpy(sub_idx).to(dev)
    te, tc = eta.index_select(0, it).cpu().numpy(), chi.index_select(0, it).cpu().numpy()
    sub = synth.subset(inp, sub_idx)
    re, rc, ae, ac = orates.forward_with_scale(sub.eps, sub.w, sub.T, sub.eta_e, sub.f,
                                               orates.Options(nquad=wl.nquad, rule=wl.rule))

    def a10(y, r, a):
        return float(np.max(np.abs(y - r) / np.maximum(np.maximum(np.abs(r), 1e-3 * a), 1e-290)))

    sampled = {"eta0": a10(te[:, :, 0], re[:, :, 0], ae[:, :, 0]), "eta1": a10(te[:, :, 1], re[:, :, 1], ae[:, :, 1]),
               "chi0": a10(tc[:, :, 0], rc[:, :, 0], ac[:, :, 0]), "chi1": a10(tc[:, :, 1], rc[:, :, 1], ac[:, :, 1]),
               "zones": len(sub_idx)}

    nv = vtx.task_values(wl.ne, 3)
    out = {"lattice": f"{nt} x {nh} nodes, d ln T = {dlnT}, d eta_e = {deta}, over the workload's range",
           "table_bytes": table.numel() * 8, "build_ms": ev[0].elapsed_time(ev[1]),
           "zones_per_launch": nz, "interp_launch_ms": t, "direct_forward_launch_ms": t_direct_ms,
           "bytes_read_per_launch": nz * (4 * nv * 8 + 16 + 1008), "bytes_written_per_launch": nz * 2016,
           "rel_err_vs_oracle_sampled": sampled,
           "l0_err_vs_direct_all_zones": {"eta0": err(eta, e0), "chi0": err(chi, c0)}}
    out["read_GBps"] = out["bytes_read_per_launch"] / (t * 1e-3) / 1e9
    del table, eta, chi, e0, c0
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=sorted(synth.WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["mixed", "fp64"])
    ap.add_argument("--fp64-steps", type=int, default=2, help="steps of the FP64 comparison run (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-errors", action="store_true")
    ap.add_argument("--stream-steps", type=int, default=2,
                    help="steps of the pinned-host streaming run, PCIe included (0: skip)")
    ap.add_argument("--fused-steps", type=int, default=2,
                    help="steps with forward and backward fused in one call per chunk (0: skip)")
    ap.add_argument("--tabulated-launches", type=int, default=3,
                    help="timed launches of the tabulated comparison over one chunk (0: skip)")
    ap.add_argument("--positron-steps", type=int, default=2,
                    help="steps of the run with neutrino-positron scattering added (0: skip)")
    ap.add_argument("--jacobian-launches", type=int, default=3,
                    help="timed launches of the explicit Jacobian over one chunk (0: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="also run one device-to-device copy of BYTES (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures a single GPU: run it with --gpus 1. The rates need no communication; "
              "more GPUs would each take a block of rays.", file=sys.stderr)
        sys.exit(2)

    import torch
    wl = synth.WORKLOADS[args.workload]
    precision = args.precision or wl.precision
    print(f"[bench] drawing workload {wl.name}: {wl.nzones} zones, NE={wl.ne}, n={wl.nquad}", file=sys.stderr,
          flush=True)
    inp = synth.make_inputs(wl.name)
    if args.copy_calibration > 0:
        n = args.copy_calibration // 8
        src = torch.arange(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {n * 8} bytes read, {n * 8} bytes written", file=sys.stderr, flush=True)
        del src, dst
    run = Runner(inp, wl, precision, wl.chunks)
    print(f"[bench] {precision}: warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    t_step = run.timed(args.steps, args.warmup)
    units = wl.nzones * wl.ne * wl.ne
    value = units / t_step
    t_fwd, t_bwd, zl = run.launch_times()
    errors = None if args.no_errors else sampled_errors(inp, run, wl)
    streaming = None
    if args.stream_steps > 0:
        print(f"[bench] streaming from pinned host memory: {args.stream_steps} steps", file=sys.stderr, flush=True)
        streaming = streaming_leg(run, units, args.stream_steps, 1)
    # after the streaming leg: it compares its outputs with this run's separate-call ones
    fused = None
    if args.fused_steps > 0:
        print(f"[bench] fused forward+backward: {args.fused_steps} steps", file=sys.stderr, flush=True)
        tf = run.timed_fused(args.fused_steps, 1)
        fused = {"value": units / tf, "unit": "zone*(eps,eps')/s", "ms_per_step": tf * 1e3,
                 "note": "vtx_rates_forward_backward: one call per chunk computes eta, chi and the VJP; "
                         "for callers holding g_eta, g_chi before the forward values"}
    del run
    torch.cuda.empty_cache()

    # roofline of the dominant kernel (backward): algorithmic FLOPs per launch / launch time
    dom_ms, dom_bwd = (t_bwd, True) if t_bwd >= t_fwd else (t_fwd, False)
    flops = algorithmic_flops_per_zone(wl.ne, wl.nquad, dom_bwd) * zl
    achieved = flops / (dom_ms * 1e-3) / 1e12
    tag = f"rates_{'backward' if dom_bwd else 'forward'}_{precision}_{wl.name}"
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS[precision], "unit": "TFLOP/s",
            "frac": achieved / PEAK_TFLOPS[precision], "traffic": traffic_from_profiles(tag),
            "kernel": tag, "launch_ms": dom_ms, "zones_per_launch": zl,
            "valu_issue": valu_issue_from_profiles(tag),
            "fwd_launch_ms": t_fwd, "bwd_launch_ms": t_bwd}

    fp64 = None
    if precision == "mixed" and args.fp64_steps > 0:
        print(f"[bench] fp64 comparison: {args.fp64_steps} steps", file=sys.stderr, flush=True)
        run64 = Runner(inp, wl, "fp64", wl.chunks)
        t64 = run64.timed(args.fp64_steps, 1)
        e64 = None if args.no_errors else sampled_errors(inp, run64, wl)
        del run64
        torch.cuda.empty_cache()
        fp64 = {"value": units / t64, "ms_per_step": t64 * 1e3, "speedup_mixed_over_fp64": t64 / t_step,
                "rel_err": e64}

    positron = None
    if args.positron_steps > 0:
        print(f"[bench] with neutrino-positron scattering: {args.positron_steps} steps", file=sys.stderr, flush=True)
        runp = Runner(inp, wl, precision, wl.chunks, processes=7)
        tp = runp.timed(args.positron_steps, 1)
        pf, pb, _ = runp.launch_times()
        positron = {"value": units / tp, "unit": "zone*(eps,eps')/s", "ms_per_step": tp * 1e3,
                    "fwd_launch_ms": pf, "bwd_launch_ms": pb,
                    "note": "all three processes (nu-e-, nu-e+ scattering, pair), same units"}
        del runp
        torch.cuda.empty_cache()

    tabulated = None
    if args.tabulated_launches > 0:
        print(f"[bench] tabulated kernels: {args.tabulated_launches} launches", file=sys.stderr, flush=True)
        tabulated = tabulated_leg(inp, wl, precision, args.tabulated_launches, t_fwd)

    jac = None
    if args.jacobian_launches > 0:
        print(f"[bench] explicit Jacobian: {args.jacobian_launches} launches", file=sys.stderr, flush=True)
        jac = jacobian_leg(inp, wl, precision, args.jacobian_launches)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(wl)

    line = {
        "metric": "zone*(eps,eps') kernel evals/sec fwd+bwd", "value": value, "unit": "zone*(eps,eps')/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_step * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.rays} rays x {wl.radial} zones, NE={wl.ne}, {wl.nquad}-node "
                               f"{wl.rule} rule, {precision}, fwd+bwd, {wl.chunks} chunks, inputs resident in HBM",
                   "zones": wl.nzones, "ne": wl.ne, "nquad": wl.nquad, "precision": precision},
        "rel_err_vs_oracle": errors, "fp64": fp64, "roofline": roof, "cpu_baseline": cpu,
        "streaming_pcie": streaming, "jacobian": jac, "with_positron_scattering": positron,
        "fused_forward_backward": fused, "tabulated": tabulated,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
