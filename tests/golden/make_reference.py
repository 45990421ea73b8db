"""Write the stored oracle references of the full-size parity tests and the benchmark's
error report: tests/golden/ref_<workload>.npz.

For each workload below, the FP64 oracle (oracle/, same rule as the library) is run on a
seeded sample of zones stratified over (T, eta_e) (paper_1404_1719_amd.synth.
sample_zones_stratified: the extreme zones, a share from the corner eta_e > 30, T < 2 MeV, the
rest spread over an 8 x 8 grid), forward on the whole sample and backward on a stratified
sub-sample, with the upstream gradients of synth.pooled_gradients (zone z takes pool row
z mod 4099, so a full-size run draws them by a gather on the device).

Stored: idx, the zones' T and eta_e, eta, chi (float64) and the absolute scales of the
relative-error floor (float32): A_eta, A_chi, the sums of the absolute values of each output's
terms, and Aq_eta, Aq_chi, the same with every kernel taken as its absolute quadrature (|H|);
idx_b, g_T, g_eta_e, g_f (float64) and aq_g_f (float32), the absolute scale of g_f = J^T g: the
sum over outputs of |g| times the Jacobian entries taken as sums of absolute quadrature terms
(|H| in the kernels), the gradient's counterpart of Aq; and a hash of the oracle's and the
sampler's sources, which the CPU tests compare with the current files.

The cool-zone workload (lowt) gets a reference of the forward with the electron mass: a
stratified sample of 512 zones, eta, chi and their scales A (the oracle's oracle/massive.py is
in its hash).

Calls only oracle/ and the seeded input generators. Usage (about ten minutes on 8 cores):
    python tests/golden/make_reference.py [--workers 8] [--only large] [--grad-scale-only]
(--grad-scale-only adds aq_g_f to existing files written from the same oracle sources.)
"""
import argparse
import hashlib
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_1404_1719_amd import synth  # noqa: E402

# workload -> (forward sample, backward sub-sample)
PLAN = {"large": (4096, 512), "medium": (1024, 128)}
# the forward with the electron mass (no backward): workload -> forward sample
PLAN_MASS = {"lowt": 512}
GRAD_SEED = 7
SAMPLE_SEED = 0


# the oracle modules the stored values come from, and the input generator
SOURCES = ("oracle/angular.py", "oracle/grad.py", "oracle/physics.py", "oracle/rates.py", "oracle/rule.py",
           "paper_1404_1719_amd/synth.py")


def source_hash(extra=()):
    """sha256 over the sources the stored values depend on (oracle modules, input generator)."""
    h = hashlib.sha256()
    files = [os.path.join(ROOT, f) for f in SOURCES + tuple(extra)]
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def path(name):
    return os.path.join(HERE, f"ref_{name}.npz")


def samples(inp, nf, nb):
    idx = synth.sample_zones_stratified(inp, nf, SAMPLE_SEED)
    sub = synth.sample_zones_stratified(synth.subset(inp, idx), nb, SAMPLE_SEED + 1)
    return idx, idx[sub]


def _fwd(args):
    from oracle import rates as orates
    eps, w, T, E, f, nquad, rule = args
    return orates.forward_with_scale(eps, w, T, E, f, orates.Options(nquad=nquad, rule=rule), quadrature=True)


def _bwd(args):
    from oracle import grad as ograd
    from oracle import rates as orates
    eps, w, T, E, f, ge, gc, nquad, rule = args
    return ograd.vjp(eps, w, T, E, f, ge, gc, orates.Options(nquad=nquad, rule=rule))


def grad_f_scale(J, ge, gc):
    """aq_g_f[z, s', m, j] = sum over outputs (s, o, i) acting on f_m of species s' of
    |g_o(s, i)| J_abs[z, s, p, o, i, j] (p = 0: s' = s; p = 1: s' = the pair partner of s)."""
    from oracle import physics
    nz, ne = J.shape[0], J.shape[-1]
    ag = np.stack([np.abs(ge[:, :, 0]), np.abs(gc[:, :, 0]), np.abs(ge[:, :, 1]), np.abs(gc[:, :, 1])], axis=2)
    out = np.zeros((nz, 3, 2, ne))
    for s in range(3):
        for p, tgt in ((0, s), (1, physics.PARTNER[s])):
            for o in range(4):
                out[:, tgt, o // 2, :] += np.einsum("zi,zij->zj", ag[:, s, o], J[:, s, p, o])
    return out


def _gscale(args):
    from oracle import rates as orates
    eps, w, T, E, ge, gc, nquad, rule = args
    J = orates.jacobian(eps, w, T, E, orates.Options(nquad=nquad, rule=rule), absolute=True)
    return grad_f_scale(J, ge, gc)


def make(name, workers):
    wl = synth.WORKLOADS[name]
    nf, nb = PLAN[name]
    t0 = time.time()
    inp = synth.make_inputs(name)
    idx, idx_b = samples(inp, nf, nb)
    print(f"[ref] {name}: {len(idx)} forward zones, {len(idx_b)} backward zones (draw {time.time() - t0:.0f} s)",
          flush=True)
    sub, sub_b = synth.subset(inp, idx), synth.subset(inp, idx_b)
    del inp
    ge, gc = synth.pooled_gradients(idx_b, wl.ne, GRAD_SEED)
    pieces = np.array_split(np.arange(len(idx)), 8 * workers)
    pieces_b = np.array_split(np.arange(len(idx_b)), 4 * workers)
    with ProcessPoolExecutor(max_workers=workers) as ex:
        fw = ex.map(_fwd, [(sub.eps, sub.w, sub.T[p], sub.eta_e[p], sub.f[p], wl.nquad, wl.rule) for p in pieces])
        bw = ex.map(_bwd, [(sub_b.eps, sub_b.w, sub_b.T[p], sub_b.eta_e[p], sub_b.f[p], ge[p], gc[p], wl.nquad,
                            wl.rule) for p in pieces_b])
        gs = ex.map(_gscale, [(sub_b.eps, sub_b.w, sub_b.T[p], sub_b.eta_e[p], ge[p], gc[p], wl.nquad, wl.rule)
                              for p in pieces_b])
        fw, bw, gs = list(fw), list(bw), list(gs)
    eta, chi, ae, ac, qe, qc = (np.concatenate([r[k] for r in fw]) for k in range(6))
    gT, gE, gf = (np.concatenate([r[k] for r in bw]) for k in range(3))
    np.savez_compressed(path(name), workload=name, source_hash=source_hash(), grad_seed=GRAD_SEED,
                        idx=idx, T=sub.T, eta_e=sub.eta_e, eta=eta, chi=chi, a_eta=ae.astype(np.float32),
                        a_chi=ac.astype(np.float32), aq_eta=qe.astype(np.float32), aq_chi=qc.astype(np.float32),
                        idx_b=idx_b, g_T=gT, g_eta_e=gE, g_f=gf, aq_g_f=np.concatenate(gs).astype(np.float32))
    print(f"[ref] {name}: written {path(name)} ({os.path.getsize(path(name)) / 1e6:.1f} MB, "
          f"{time.time() - t0:.0f} s)", flush=True)


def add_grad_scale(name, workers):
    """Add aq_g_f to an existing reference written from the current oracle sources."""
    wl = synth.WORKLOADS[name]
    ref = load(name)
    if str(ref["source_hash"]) != source_hash():
        raise SystemExit(f"ref_{name}.npz was written from other oracle sources: regenerate it whole")
    t0 = time.time()
    sub_b = synth.subset(synth.make_inputs(name), ref["idx_b"])
    ge, gc = synth.pooled_gradients(ref["idx_b"], wl.ne, GRAD_SEED)
    pieces_b = np.array_split(np.arange(len(ref["idx_b"])), 4 * workers)
    with ProcessPoolExecutor(max_workers=workers) as ex:
        gs = list(ex.map(_gscale, [(sub_b.eps, sub_b.w, sub_b.T[p], sub_b.eta_e[p], ge[p], gc[p], wl.nquad, wl.rule)
                                   for p in pieces_b]))
    ref["aq_g_f"] = np.concatenate(gs).astype(np.float32)
    np.savez_compressed(path(name), **ref)
    print(f"[ref] {name}: aq_g_f added ({time.time() - t0:.0f} s)", flush=True)


def _fwd_mass(args):
    from oracle import rates as orates
    eps, w, T, E, f, nquad, rule = args
    return orates.forward_with_scale(eps, w, T, E, f, orates.Options(nquad=nquad, rule=rule, electron_mass=True))


def make_mass(name, workers):
    """Forward with the electron mass on a stratified sample (default processes), outputs and
    their output-level scales A."""
    wl = synth.WORKLOADS[name]
    t0 = time.time()
    inp = synth.make_inputs(name)
    idx = synth.sample_zones_stratified(inp, PLAN_MASS[name], SAMPLE_SEED)
    sub = synth.subset(inp, idx)
    del inp
    pieces = np.array_split(np.arange(len(idx)), 8 * workers)
    with ProcessPoolExecutor(max_workers=workers) as ex:
        fw = list(ex.map(_fwd_mass, [(sub.eps, sub.w, sub.T[p], sub.eta_e[p], sub.f[p], wl.nquad, wl.rule)
                                     for p in pieces]))
    eta, chi, ae, ac = (np.concatenate([r[k] for r in fw]) for k in range(4))
    np.savez_compressed(path(name), workload=name, source_hash=source_hash(("oracle/massive.py",)), idx=idx,
                        T=sub.T, eta_e=sub.eta_e, eta=eta, chi=chi, a_eta=ae.astype(np.float32),
                        a_chi=ac.astype(np.float32))
    print(f"[ref] {name}: written {path(name)} ({os.path.getsize(path(name)) / 1e6:.1f} MB, "
          f"{time.time() - t0:.0f} s)", flush=True)


def load(name):
    """The stored reference of a workload as a dict of arrays (no pickle)."""
    with np.load(path(name), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--only", default=None, choices=sorted(PLAN) + sorted(PLAN_MASS))
    ap.add_argument("--grad-scale-only", action="store_true")
    a = ap.parse_args()
    for n in PLAN:
        if a.only in (None, n):
            (add_grad_scale if a.grad_scale_only else make)(n, a.workers)
    for n in PLAN_MASS:
        if a.only in (None, n) and not a.grad_scale_only:
            make_mass(n, a.workers)
