"""Benchmark: zone x (eps, eps') kernel evaluations per second, forward + backward.

One step = forward (eta, chi) + backward (g_T, g_eta_e, g_f) over every zone of the
workload, inputs resident in HBM, in 8 chunks issued back to back on one compute stream.
Default workload: 4096 rays x 600 zones, NE = 21, 64-node rule, mixed precision (zones with
|eta_e| > 30 entirely in FP64). Prints ONE JSON line. Units: zones * NE^2 per second
(each unit covers 3 species, both processes, l = 0, 1, one forward and one backward
evaluation).

Also reported: the same step in plain FP64 (speedup of mixed over FP64, and its own roofline
entry); the maximal relative error per output against stored FP64 oracle outputs
(tests/golden/ref_<workload>.npz, written by a script that calls only the oracle) on 4,096
stratified zones forward and 512 backward, with the stratum eta_e > 30, T < 2 MeV on its own;
a roofline entry for the dominant launch; the oracle timed on the host cores on a bounded
sample; the whole step end to end with the workload in pinned host memory, streamed through
the GPU in 8 chunks (package stream.Streamer, PCIe transfers included); the mixed path with
the FP64 zone-class threshold at 64 instead of 30; the explicit Jacobian blocks over one
chunk; the tabulated comparison; all three processes; the fused forward + backward call.
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

# The paper's own performance figures: whole-application rates of the CPU code on its clusters,
# context for the numbers above, not a baseline for them (the paper gives none for the rates).
PAPER_CONTEXT = {
    "note": "whole PROMETHEUS-VERTEX application on CPU clusters; not comparable with the rates kernels",
    "node": {"value": 10.0, "unit": "GFlop/s", "hardware": "2x Intel Xeon E5540 (Nehalem), 8 cores, 2.53 GHz",
             "detail": "more than 12 % of the node's 81 GFlop/s peak, memory bound at an arithmetic intensity of "
                       "0.96 flop/byte (Sect. 3.2, Fig. 3)"},
    "system": {"value": 0.25, "unit": "PFlop/s", "hardware": "SuperMUC",
               "detail": "sustained, about 10 % of nominal peak; derived from about 35 GFlop/s per SandyBridge node "
                         "and the weak-scaling efficiency over 1-8192 nodes (Sect. 3.2)"},
}


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


def load_reference(name):
    """Stored FP64 oracle outputs of a workload's zone sample, or None (tests/golden)."""
    path = os.path.join(ROOT, "tests", "golden", f"ref_{name}.npz")
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def stored_errors(inp, run, ref, stratum=None):
    """Max relative error per output against the stored oracle outputs: forward on the
    reference's zone sample, |y - y_ref| / max(|y_ref|, floor, 1e-290): FP64 floor 1e-3 A, A the
    sum of |terms|; mixed floor 1e-2 Aq, Aq that sum with |H| kernels, the scale below which FP32
    rounding of a 64-node quadrature (about 2^-24 sqrt(8 x 64) Aq) exceeds 1e-4 of |y|;
    backward on its sub-sample for the run's pooled upstream gradients, floor 1e-3 x the mean
    magnitude of the field (g_f = K^T g sums terms of both signs; the mixed path's g_f instead
    1e-2 of its absolute-term scale aq_g_f). stratum(T, eta_e) selects
    zones reported again on their own."""
    import torch
    idx, idx_b = ref["idx"], ref["idx_b"]

    def pick(t, ix):
        return t.index_select(0, torch.from_numpy(ix).to(t.device)).cpu().numpy()

    def ferr(y, r, a, floor):
        return np.abs(y - r) / np.maximum(np.maximum(np.abs(r), floor * a.astype(np.float64)), 1e-290)

    def gerr(g, r):
        return np.abs(g - r) / np.maximum(np.abs(r), 1e-3 * np.mean(np.abs(r)) + 1e-300)

    e, c = pick(run.eta, idx), pick(run.chi, idx)

    def forward_errors(scale, floor):
        return {"eta0": ferr(e[:, :, 0], ref["eta"][:, :, 0], ref[scale + "_eta"][:, :, 0], floor),
                "eta1": ferr(e[:, :, 1], ref["eta"][:, :, 1], ref[scale + "_eta"][:, :, 1], floor),
                "chi0": ferr(c[:, :, 0], ref["chi"][:, :, 0], ref[scale + "_chi"][:, :, 0], floor),
                "chi1": ferr(c[:, :, 1], ref["chi"][:, :, 1], ref[scale + "_chi"][:, :, 1], floor)}

    # the mixed path's bar uses the quadrature-level scale Aq, the FP64 path's the output level A
    f = forward_errors("aq", 1e-2) if run.precision == "mixed" else forward_errors("a", 1e-3)
    fa = forward_errors("a", 1e-3)
    g = {k: gerr(pick(t, idx_b), ref[k]) for k, t in (("g_T", run.gT), ("g_eta_e", run.gE), ("g_f", run.gf))}
    if run.precision == "mixed" and "aq_g_f" in ref:
        # g_f sums kernel entries of both signs: the mixed floor is 1e-2 of its absolute-term scale
        g["g_f"] = ferr(pick(run.gf, idx_b), ref["g_f"], ref["aq_g_f"], 1e-2)
    out = {k: float(v.max()) for k, v in {**f, **g}.items()}
    out["floor"] = "1e-2 Aq (sum of |terms| with |H| kernels)" if run.precision == "mixed" else "1e-3 A"
    if run.precision == "mixed":
        n_all = sum(v.size for v in fa.values())
        out["output_level_floor"] = {**{k: float(v.max()) for k, v in fa.items()},
                                     "entries_above_1e-4": sum(int((v > 1e-4).sum()) for v in fa.values()),
                                     "entries": n_all}
    out["zones_forward"], out["zones_backward"] = int(idx.size), int(idx_b.size)
    if stratum is not None:
        sf, sb = stratum(inp.T[idx], inp.eta_e[idx]), stratum(inp.T[idx_b], inp.eta_e[idx_b])
        out["stratum"] = {**{k: float(v[sf].max(initial=0.0)) for k, v in f.items()},
                          **{k: float(v[sb].max(initial=0.0)) for k, v in g.items()},
                          "zones_forward": int(sf.sum()), "zones_backward": int(sb.sum())}
    return out


def corner(T, eta_e):
    """The stratum of high degeneracy at low temperature: eta_e > 30, T < 2 MeV."""
    return (eta_e > 30.0) & (T < 2.0)


class Runner:
    """Device-resident buffers of one workload and the chunked two-stream step."""

    def __init__(self, inp, wl, precision, chunks, processes=3, eta_fp64=30.0, grad_seed=7):
        import torch
        from paper_1404_1719_amd import vtx
        self.torch, self.vtx = torch, vtx
        dev = torch.device("cuda:0")
        self.grid = vtx.GridHandle(inp.eps, inp.w)
        self.precision = precision
        self.opts = vtx.make_opts(precision, wl.nquad, wl.rule, processes, eta_fp64=eta_fp64)
        self.nz, self.ne = inp.T.shape[0], wl.ne
        self.T = torch.from_numpy(inp.T).to(dev)
        self.E = torch.from_numpy(inp.eta_e).to(dev)
        self.f = torch.from_numpy(inp.f).to(dev)
        shp = (self.nz, 3, 2, self.ne)
        # upstream gradients: zone z takes row z mod 4099 of a seeded pool (synth.pooled_gradients),
        # the rows the stored oracle reference used
        pe, pc = (torch.from_numpy(a).to(dev) for a in synth.gradient_pool(self.ne, grad_seed))
        rows = torch.arange(self.nz, device=dev) % pe.shape[0]
        self.g_eta, self.g_chi = pe.index_select(0, rows), pc.index_select(0, rows)
        del pe, pc, rows
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


def streaming_leg(inp, run, units, steps, warmup):
    """Whole step end to end with the workload in pinned host memory, streamed through the GPU
    in the workload's chunks by the package's stream.Streamer (PCIe transfers included): its
    outputs are compared with the resident run's, bit for bit."""
    torch = run.torch
    from paper_1404_1719_amd import stream
    st = stream.Streamer(run.grid, run.opts, run.nz, chunks=len(run.chunks))
    for k, t in (("T", run.T), ("eta_e", run.E), ("f", run.f), ("g_eta", run.g_eta), ("g_chi", run.g_chi)):
        st.host[k].copy_(t)
    for _ in range(warmup):
        st.step()
    st.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st.step()
    st.synchronize()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / max(steps, 1)
    same = all(bool(torch.equal(st.host[k], x.cpu())) for k, x in
               (("eta", run.eta), ("chi", run.chi), ("g_T", run.gT), ("g_eta_e", run.gE), ("g_f", run.gf)))
    out = {"value": units / t, "unit": "zone*(eps,eps')/s", "ms_per_step": t * 1e3, "steps": steps,
           "chunks": len(st.chunks), "bytes_h2d": st.bytes_h2d, "bytes_to_host": st.bytes_d2h,
           "pcie_GBps": (st.bytes_h2d + st.bytes_d2h) / t / 1e9, "outputs_equal_resident_run": same,
           "note": "paper_1404_1719_amd.stream.Streamer: pinned host arrays; inputs by DMA copies into 2 device "
                   "buffer sets; forward and backward of a chunk on two compute streams at once; outputs "
                   "written by the kernels into the mapped host arrays"}
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


def mass_leg(launches):
    """The forward with the electron mass (FP64) on the cool-zone workload, whose regime it is
    for, beside the massless FP64 forward on the same zones: launch times with HIP events on
    the launch stream, forward-only rates in the headline's units."""
    import torch
    from paper_1404_1719_amd import vtx
    wl = synth.WORKLOADS["lowt"]
    inp = synth.make_inputs("lowt")
    dev = torch.device("cuda:0")
    grid = vtx.GridHandle(inp.eps, inp.w)
    opts = vtx.make_opts("fp64", wl.nquad, wl.rule)
    T, E, f = (torch.from_numpy(a).to(dev) for a in (inp.T, inp.eta_e, inp.f))
    eta, chi = torch.empty_like(f), torch.empty_like(f)
    s = torch.cuda.Stream(device=dev)
    s.wait_stream(torch.cuda.current_stream())
    out = {}
    for name, fn in (("mass", vtx.forward_mass), ("massless", vtx.forward)):
        ms = []
        with torch.cuda.stream(s):
            fn(grid, opts, T, E, f, eta, chi, stream=s)
            for _ in range(launches):
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
                ev[0].record(s)
                fn(grid, opts, T, E, f, eta, chi, stream=s)
                ev[1].record(s)
                ms.append(ev)
        s.synchronize()
        out[name] = float(np.mean([a.elapsed_time(b) for a, b in ms]))
        out[name + "_finite"] = bool(torch.isfinite(eta).all() and torch.isfinite(chi).all())
    del T, E, f, eta, chi
    torch.cuda.empty_cache()
    units = wl.nzones * wl.ne * wl.ne
    return {"workload": f"{wl.name}: {wl.nzones} zones, NE={wl.ne} bins {wl.emin:g}-{wl.emax:g} MeV, "
                        f"T ~ U{wl.t_range} MeV, eta_e ~ U{wl.eta_range}, {wl.nquad}-node panel rule, FP64, forward",
            "value": units / (out["mass"] * 1e-3), "unit": "zone*(eps,eps')/s (forward only)",
            "launch_ms": out["mass"], "massless_fp64_launch_ms": out["massless"],
            "cost_vs_massless": out["mass"] / out["massless"], "outputs_finite": out["mass_finite"],
            "kernel": "rates_mass_kernel"}


def newton_leg(inp, wl, precision, nrays):
    """Newton step of the radial sweep over nrays rays (at most the workload's) x the workload's
    radial zones (the first zones): the rates and their explicit blocks (vtx_rates_jacobian), the
    system (vtx_ray_system) and the block-tridiagonal solve (vtx_ray_solve), each timed with HIP
    events on its stream. Time step and radial coupling on the rates' scale (dt = 1/kappa,
    lo, up ~ kappa U(0, 1/2), kappa the median opacity). Algorithmic work of the solve: per zone
    one Gauss-Jordan inversion of a 6 NE block (2 nb^3 flop) and three block-vector products
    (6 nb^2); the system writes nb^2 + nb doubles per zone and reads the 24 NE^2 of the blocks."""
    import torch
    from paper_1404_1719_amd import vtx
    nzr = wl.radial
    nrays = min(nrays, wl.rays)
    nz = nrays * nzr
    ne, nb = wl.ne, 6 * wl.ne
    dev = torch.device("cuda:0")
    grid = vtx.GridHandle(inp.eps, inp.w)
    opts = vtx.make_opts(precision, wl.nquad, wl.rule)
    T = torch.from_numpy(inp.T[:nz]).to(dev)
    E = torch.from_numpy(inp.eta_e[:nz]).to(dev)
    f = torch.from_numpy(inp.f[:nz]).to(dev)
    g = torch.Generator(device=dev)
    g.manual_seed(synth.SEED_BASE + 6000)
    f_n = (f * (1 + 0.01 * torch.randn(f.shape, dtype=torch.float64, device=dev, generator=g))).clamp(0, 1)
    s = torch.cuda.Stream(device=dev)
    s.wait_stream(torch.cuda.current_stream())
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    with torch.cuda.stream(s):
        ev[0].record(s)
        jac, eta, chi = vtx.jacobian(grid, opts, T, E, stream=s, f=f)
        ev[1].record(s)
        kappa = torch.median(chi[:, :, 0])
        lo = kappa * 0.5 * torch.rand((nz, nb), dtype=torch.float64, device=dev, generator=g)
        up = kappa * 0.5 * torch.rand((nz, nb), dtype=torch.float64, device=dev, generator=g)
        dt = 1.0 / float(kappa.item())
        D = torch.empty((nz, nb, nb), dtype=torch.float64, device=dev)
        rhs = torch.empty((nz, nb), dtype=torch.float64, device=dev)
        ev[2].record(s)
        vtx.ray_system(ne, nrays, nzr, dt, jac, f, f_n, f_n, eta, chi, lo, up, D=D, rhs=rhs, stream=s)
        ev[3].record(s)
        vtx.ray_solve(nrays, nzr, lo, D, up, rhs, stream=s)
        ev[4].record(s)
    s.synchronize()
    finite = bool(torch.isfinite(rhs).all().item())
    t_rates, t_sys, t_solve = ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3]), ev[3].elapsed_time(ev[4])
    flops = nz * (2.0 * nb ** 3 + 6.0 * nb ** 2)
    sys_bytes = nz * 8.0 * (nb * nb + nb + 24 * ne * ne + 10 * nb)
    solve_bytes = nz * 8.0 * (3 * nb * nb + 6 * nb)
    out = {"rays": nrays, "zones_per_ray": nzr, "block": nb, "rates_and_blocks_ms": t_rates,
           "system_ms": t_sys, "system_GBps": sys_bytes / (t_sys * 1e-3) / 1e9,
           "solve_ms": t_solve, "solve_TFLOPs": flops / (t_solve * 1e-3) / 1e12,
           "solve_frac_fp64_peak": flops / (t_solve * 1e-3) / 78.6e12,
           "solve_GBps": solve_bytes / (t_solve * 1e-3) / 1e9, "solution_finite": finite,
           "note": "one Newton update of the BDF2 radial system along each ray; solve = block "
                   "elimination with Gauss-Jordan inversion of each diagonal block in the registers of "
                   "one 1024-lane workgroup per ray"}
    del jac, eta, chi, D, rhs, lo, up, T, E, f, f_n
    torch.cuda.empty_cache()
    return out


def tabulated_leg(inp, wl, precision, launches, t_direct_ms, ref):
    """Tabulated comparison point: task values on a (ln T, eta_e) lattice over the workload's
    range (built by the library), interpolated per zone over one chunk, against the direct
    forward. Errors: against the stored FP64 oracle outputs on the reference zones inside the
    chunk, with the floor of the direct path; and over every zone of the chunk for the l = 0
    outputs (which do not cancel), against the library's direct forward,
    |y_tab - y| / max(|y|, 1e-3 max over the bins of the same output)."""
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

    sampled = None
    if ref is not None:
        keep = ref["idx"] < nz
        sub_idx = ref["idx"][keep]
        it = torch.from_numpy(sub_idx).to(dev)
        te, tc = eta.index_select(0, it).cpu().numpy(), chi.index_select(0, it).cpu().numpy()
        re, rc = ref["eta"][keep], ref["chi"][keep]
        ae, ac = ref["a_eta"][keep].astype(np.float64), ref["a_chi"][keep].astype(np.float64)

        def a10(y, r, a):
            return float(np.max(np.abs(y - r) / np.maximum(np.maximum(np.abs(r), 1e-3 * a), 1e-290)))

        sampled = {"eta0": a10(te[:, :, 0], re[:, :, 0], ae[:, :, 0]),
                   "eta1": a10(te[:, :, 1], re[:, :, 1], ae[:, :, 1]),
                   "chi0": a10(tc[:, :, 0], rc[:, :, 0], ac[:, :, 0]),
                   "chi1": a10(tc[:, :, 1], rc[:, :, 1], ac[:, :, 1]), "zones": int(sub_idx.size)}

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


def roofline(wl, precision, t_fwd, t_bwd, zl, f64_share=None):
    """Roofline entry of the dominant launch (the backward call of a chunk): algorithmic FLOPs
    per launch / its HIP-event duration. In the mixed path that call runs two kernels, one per
    zone class (FP32 up to |eta_e| = eta_fp64, FP64 above), and its duration is their sum. Its
    peak is then the one its arithmetic can reach: the share f of zones in the FP64 class runs
    the same algorithm at the FP64 vector rate, so the call's attainable rate is
    1 / ((1 - f) / P32 + f / P64) (f from the workload's eta_e); the FP32 peak is reported
    beside it."""
    dom_ms, dom_bwd = (t_bwd, True) if t_bwd >= t_fwd else (t_fwd, False)
    flops = algorithmic_flops_per_zone(wl.ne, wl.nquad, dom_bwd) * zl
    achieved = flops / (dom_ms * 1e-3) / 1e12
    tag = f"rates_{'backward' if dom_bwd else 'forward'}_{precision}_{wl.name}"
    peak = PEAK_TFLOPS[precision]
    out = {"bound": "alu", "achieved": achieved, "unit": "TFLOP/s"}
    if precision == "mixed" and f64_share is not None:
        peak = 1.0 / ((1.0 - f64_share) / PEAK_TFLOPS["mixed"] + f64_share / PEAK_TFLOPS["fp64"])
        out["peak_derivation"] = (f"{f64_share:.4f} of the zones in the FP64 class: "
                                  f"1 / ((1 - f) / {PEAK_TFLOPS['mixed']} + f / {PEAK_TFLOPS['fp64']})")
        out["peak_fp32"] = PEAK_TFLOPS["mixed"]
        out["frac_of_fp32_peak"] = achieved / PEAK_TFLOPS["mixed"]
    out.update({"peak": peak, "frac": achieved / peak, "traffic": traffic_from_profiles(tag), "kernel": tag,
                "launch_ms": dom_ms, "zones_per_launch": zl, "valu_issue": valu_issue_from_profiles(tag),
                "fwd_launch_ms": t_fwd, "bwd_launch_ms": t_bwd})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=sorted(synth.WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["mixed", "fp64"])
    ap.add_argument("--fp64-steps", type=int, default=2, help="steps of the FP64 comparison run (0: skip)")
    ap.add_argument("--eta-fp64", type=float, default=30.0,
                    help="mixed path: zones with |eta_e| above this run in FP64 (default 30, capped at 64)")
    ap.add_argument("--threshold64-steps", type=int, default=2,
                    help="steps of the mixed run with the FP64 zone-class threshold at 64 (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-errors", action="store_true")
    ap.add_argument("--stream-steps", type=int, default=2,
                    help="steps of the end-to-end run from pinned host memory, PCIe included (0: skip)")
    ap.add_argument("--fused-steps", type=int, default=2,
                    help="steps with forward and backward fused in one call per chunk (0: skip)")
    ap.add_argument("--tabulated-launches", type=int, default=3,
                    help="timed launches of the tabulated comparison over one chunk (0: skip)")
    ap.add_argument("--positron-steps", type=int, default=2,
                    help="steps of the run with neutrino-positron scattering added (0: skip)")
    ap.add_argument("--newton-rays", type=int, default=256,
                    help="rays of the Newton-step leg (radial zones of the workload each; 0: skip)")
    ap.add_argument("--jacobian-launches", type=int, default=3,
                    help="timed launches of the explicit Jacobian over one chunk (0: skip)")
    ap.add_argument("--mass-launches", type=int, default=3,
                    help="launches of the forward with the electron mass on the cool-zone workload (0: skip)")
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
    ref = None if args.no_errors else load_reference(wl.name)
    run = Runner(inp, wl, precision, wl.chunks, eta_fp64=args.eta_fp64)
    print(f"[bench] {precision}: warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    t_step = run.timed(args.steps, args.warmup)
    units = wl.nzones * wl.ne * wl.ne
    value = units / t_step
    t_fwd, t_bwd, zl = run.launch_times()
    errors = None if ref is None else stored_errors(inp, run, ref, corner)
    streaming = None
    if args.stream_steps > 0:
        print(f"[bench] end to end from pinned host memory: {args.stream_steps} steps", file=sys.stderr, flush=True)
        streaming = streaming_leg(inp, run, units, args.stream_steps, 1)
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

    f64_share = float(np.mean(np.abs(inp.eta_e) > min(args.eta_fp64, 64.0))) if precision == "mixed" else None
    roof = roofline(wl, precision, t_fwd, t_bwd, zl, f64_share)

    fp64 = None
    if precision == "mixed" and args.fp64_steps > 0:
        print(f"[bench] fp64 comparison: {args.fp64_steps} steps", file=sys.stderr, flush=True)
        run64 = Runner(inp, wl, "fp64", wl.chunks)
        t64 = run64.timed(args.fp64_steps, 1)
        f64, b64, z64 = run64.launch_times()
        e64 = None if ref is None else stored_errors(inp, run64, ref, corner)
        del run64
        torch.cuda.empty_cache()
        fp64 = {"value": units / t64, "ms_per_step": t64 * 1e3, "speedup_mixed_over_fp64": t64 / t_step,
                "rel_err": e64, "roofline": roofline(wl, "fp64", f64, b64, z64)}

    thr64 = None
    if precision == "mixed" and args.threshold64_steps > 0:
        print(f"[bench] mixed with the FP64 zone-class threshold at 64: {args.threshold64_steps} steps",
              file=sys.stderr, flush=True)
        r64 = Runner(inp, wl, "mixed", wl.chunks, eta_fp64=64.0)
        tt = r64.timed(args.threshold64_steps, 1)
        et = None if ref is None else stored_errors(inp, r64, ref, lambda T, e: e > 30.0)
        del r64
        torch.cuda.empty_cache()
        thr64 = {"value": units / tt, "ms_per_step": tt * 1e3, "rel_err": et,
                 "note": "FP32 for zones up to |eta_e| = 64 (the headline runs zones above 30 in FP64); "
                         "'stratum' is eta_e > 30, the zones that change class"}

    positron = None
    if args.positron_steps > 0:
        print(f"[bench] with neutrino-positron scattering: {args.positron_steps} steps", file=sys.stderr, flush=True)
        runp = Runner(inp, wl, precision, wl.chunks, processes=7, eta_fp64=args.eta_fp64)
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
        tabulated = tabulated_leg(inp, wl, precision, args.tabulated_launches, t_fwd, ref)

    jac = None
    if args.jacobian_launches > 0:
        print(f"[bench] explicit Jacobian: {args.jacobian_launches} launches", file=sys.stderr, flush=True)
        jac = jacobian_leg(inp, wl, precision, args.jacobian_launches)

    newton = None
    if args.newton_rays > 0:
        print(f"[bench] Newton step of the radial sweep: {args.newton_rays} rays", file=sys.stderr, flush=True)
        newton = newton_leg(inp, wl, precision, args.newton_rays)

    mass = None
    if args.mass_launches > 0:
        print(f"[bench] forward with the electron mass: {args.mass_launches} launches", file=sys.stderr, flush=True)
        mass = mass_leg(args.mass_launches)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(wl)

    mode = (f"FP32 quadrature bulk, FP64 contractions; zones with |eta_e| > {min(args.eta_fp64, 64.0):g} entirely in FP64"
            if precision == "mixed" else "FP64")
    line = {
        "metric": "zone*(eps,eps') kernel evals/sec fwd+bwd", "value": value, "unit": "zone*(eps,eps')/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_step * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.rays} rays x {wl.radial} zones, NE={wl.ne}, {wl.nquad}-node "
                               f"{wl.rule} rule, {precision}, fwd+bwd, {wl.chunks} chunks, inputs resident in HBM",
                   "zones": wl.nzones, "ne": wl.ne, "nquad": wl.nquad, "precision": precision,
                   "eta_fp64": args.eta_fp64 if precision == "mixed" else None, "arithmetic": mode,
                   "streaming": "value: inputs resident in HBM; end_to_end_streamed: host memory, "
                                f"{wl.chunks} stream-overlapped chunks, PCIe included"},
        "rel_err_vs_oracle": errors, "fp64": fp64, "roofline": roof, "cpu_baseline": cpu,
        "end_to_end_streamed": streaming, "threshold_64": thr64, "jacobian": jac, "newton_step": newton,
        "with_positron_scattering": positron, "fused_forward_backward": fused, "tabulated": tabulated,
        "electron_mass": mass,
        "paper_context": PAPER_CONTEXT,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
