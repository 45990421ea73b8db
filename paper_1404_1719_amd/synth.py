"""Seeded synthetic workloads: energy grid, zone states and neutrino distributions.

This module is shared by the test suite, the benchmark and the CPU oracle's callers.
It holds no part of the rate computation itself: it only draws inputs.

Workloads (named by shape; all draw order fixed as T, eta_e, a_s, noise, h):

* ``small``   : 1 ray x 64 radial zones, NE = 12 log bins 2-300 MeV, T ~ U(3, 30) MeV,
                eta_e ~ U(0, 20), a_s = mu_nu/T ~ U(-2, 10), no noise, 32 nodes, Gauss-Laguerre rule.
* ``medium``  : 256 rays x 400 zones, NE = 21 log bins 2-380 MeV, T ~ U(1, 40), eta_e ~ U(0, 40),
                a_s ~ U(-2, 15), 5 % multiplicative log-normal noise on f0, 48 nodes, panel rule.
* ``large``   : 4096 rays x 600 zones, NE = 21, T ~ U(0.5, 60), eta_e ~ U(0, 60), a_s ~ U(-2, 15),
                5 % noise, 64 nodes, panel rule (one GPU's share of a 3-D model).
* ``lowt``    : 256 rays x 400 zones, NE = 21 log bins 0.5-300 MeV, T ~ U(0.2, 8), eta_e ~ U(-2, 30),
                a_s ~ U(-2, 10), 5 % noise, 48 nodes, panel rule: the cool, outer zones where the
                electron mass (0.511 MeV) is not small against T and the lowest bins, the regime
                of the rates with the electron mass.

Energy grid: NE + 1 geometric bin edges e_0..e_NE, centres eps_i = sqrt(e_i e_{i+1}) and
bin volumes w_i = (e_{i+1}^3 - e_i^3)/3 [MeV^3], the measure of the eps'^2 d eps' phase-space
integral over bin i (the paper writes intensities with the (2 pi hbar c)^3 phase-space
normalisation, Sect. 2.1).

Neutrino distribution per zone, species s and bin i:
  f0 = 1 / (exp(eps_i/T - a_s) + 1), optionally f0 <- clip(f0 * exp(0.05 N(0,1)), 0, 1);
  f1 = h f0 (1 - f0) with h ~ U(0, 1/3) per (zone, species), so that f0 + 3 mu f1 stays in [0, 1].
Layout: f[zone][species][moment][bin], species order (nu_e, anti-nu_e, nu_x).
"""
from __future__ import annotations

import dataclasses
import numpy as np

NSPECIES = 3
SEED_BASE = 14041719


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    seed_index: int
    rays: int
    radial: int
    ne: int
    emin: float
    emax: float
    t_range: tuple
    eta_range: tuple
    a_range: tuple
    noise: float
    nquad: int
    rule: str          # "laguerre" or "panel"
    precision: str     # default arithmetic of the workload: "fp64" or "mixed"
    chunks: int = 1

    @property
    def nzones(self) -> int:
        return self.rays * self.radial


WORKLOADS = {
    "small": Workload("small", 1, 1, 64, 12, 2.0, 300.0, (3.0, 30.0), (0.0, 20.0), (-2.0, 10.0),
                      0.0, 32, "laguerre", "fp64"),
    "medium": Workload("medium", 2, 256, 400, 21, 2.0, 380.0, (1.0, 40.0), (0.0, 40.0), (-2.0, 15.0),
                       0.05, 48, "panel", "fp64"),
    "medium-mixed": Workload("medium-mixed", 3, 256, 400, 21, 2.0, 380.0, (1.0, 40.0), (0.0, 40.0),
                             (-2.0, 15.0), 0.05, 48, "panel", "mixed"),
    "medium-grad": Workload("medium-grad", 4, 256, 400, 21, 2.0, 380.0, (1.0, 40.0), (0.0, 40.0),
                            (-2.0, 15.0), 0.05, 48, "panel", "fp64"),
    "large": Workload("large", 5, 4096, 600, 21, 2.0, 380.0, (0.5, 60.0), (0.0, 60.0), (-2.0, 15.0),
                      0.05, 64, "panel", "mixed", chunks=8),
    "lowt": Workload("lowt", 6, 256, 400, 21, 0.5, 300.0, (0.2, 8.0), (-2.0, 30.0), (-2.0, 10.0),
                     0.05, 48, "panel", "fp64"),
}


def energy_grid(ne: int, emin: float, emax: float):
    """Geometric edges, centres eps_i = sqrt(e_i e_{i+1}) and volumes w_i = (e_{i+1}^3 - e_i^3)/3."""
    edges = np.geomspace(emin, emax, ne + 1)
    eps = np.sqrt(edges[1:] * edges[:-1])
    w = (edges[1:] ** 3 - edges[:-1] ** 3) / 3.0
    return eps, w


@dataclasses.dataclass
class ZoneInputs:
    eps: np.ndarray      # [NE]
    w: np.ndarray        # [NE]
    T: np.ndarray        # [Z]   MeV
    eta_e: np.ndarray    # [Z]   electron degeneracy mu_e / T
    f: np.ndarray        # [Z, 3, 2, NE]


def draw_zones(nzones: int, ne: int, eps: np.ndarray, t_range, eta_range, a_range, noise, seed):
    """Draw zone states and distributions in the fixed order T, eta_e, a_s, noise, h."""
    rng = np.random.Generator(np.random.PCG64(seed))
    T = rng.uniform(t_range[0], t_range[1], nzones)
    eta_e = rng.uniform(eta_range[0], eta_range[1], nzones)
    a = rng.uniform(a_range[0], a_range[1], (nzones, NSPECIES))
    z = eps[None, None, :] / T[:, None, None] - a[:, :, None]
    with np.errstate(over="ignore"):
        f0 = 1.0 / (np.exp(z) + 1.0)
    if noise > 0.0:
        f0 = np.clip(f0 * np.exp(noise * rng.standard_normal(f0.shape)), 0.0, 1.0)
    h = rng.uniform(0.0, 1.0 / 3.0, (nzones, NSPECIES))
    f1 = h[:, :, None] * f0 * (1.0 - f0)
    f = np.stack([f0, f1], axis=2)  # [Z, 3, 2, NE]
    return T, eta_e, np.ascontiguousarray(f)


def make_inputs(workload: str | Workload, nzones: int | None = None) -> ZoneInputs:
    """Full (or first-``nzones``) seeded inputs of a named workload.

    Drawing a prefix uses the same stream as the full workload only for the T array;
    callers that need bit-identical subsets of a full-size workload draw it whole and
    slice (``subset``)."""
    wl = WORKLOADS[workload] if isinstance(workload, str) else workload
    eps, w = energy_grid(wl.ne, wl.emin, wl.emax)
    nz = wl.nzones if nzones is None else nzones
    T, eta_e, f = draw_zones(nz, wl.ne, eps, wl.t_range, wl.eta_range, wl.a_range, wl.noise,
                             SEED_BASE + wl.seed_index)
    return ZoneInputs(eps, w, T, eta_e, f)


def subset(inp: ZoneInputs, idx) -> ZoneInputs:
    idx = np.asarray(idx)
    return ZoneInputs(inp.eps, inp.w, inp.T[idx].copy(), inp.eta_e[idx].copy(),
                      np.ascontiguousarray(inp.f[idx]))


def sample_zones(inp: ZoneInputs, count: int, seed: int = 0):
    """Indices of a seeded zone sample that always holds the min-T, max-T and max-eta_e zones."""
    nz = inp.T.shape[0]
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 1000 + seed))
    forced = {int(np.argmin(inp.T)), int(np.argmax(inp.T)), int(np.argmax(inp.eta_e))}
    rest = rng.choice(nz, size=min(nz, count + 3), replace=False)
    out = list(forced)
    for r in rest:
        if len(out) >= min(count, nz):
            break
        if int(r) not in forced:
            out.append(int(r))
    return np.array(sorted(out), dtype=np.int64)


def random_gradients(nzones: int, ne: int, seed: int):
    """Seeded upstream gradients g_eta, g_chi of shape [Z, 3, 2, NE] (unit normal entries)."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 2000 + seed))
    g_eta = rng.standard_normal((nzones, NSPECIES, 2, ne))
    g_chi = rng.standard_normal((nzones, NSPECIES, 2, ne))
    return g_eta, g_chi


def sample_zones_stratified(inp: ZoneInputs, count: int, seed: int = 0, corner_share: float = 0.125,
                            cells: int = 8):
    """Indices of a seeded zone sample stratified over (T, eta_e).

    Always holds the min-T, max-T, min-eta_e and max-eta_e zones; then about ``corner_share``
    of the sample from the corner of high degeneracy at low temperature (eta_e > 30 and T < 2
    MeV, where the Fermi-Dirac factors are most extreme); the rest spread evenly over a
    ``cells`` x ``cells`` grid of T (geometric bins) and eta_e (uniform bins) over the zones'
    range, drawn at random inside each cell. Sorted, without repeats."""
    nz = inp.T.shape[0]
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 1500 + seed))
    chosen = []
    seen = set()

    def take(cands, k):
        cands = np.asarray(cands)
        if cands.size == 0 or k <= 0:
            return
        picks = rng.permutation(cands)
        n = 0
        for c in picks:
            c = int(c)
            if c not in seen:
                seen.add(c)
                chosen.append(c)
                n += 1
                if n >= k:
                    break

    for c in (np.argmin(inp.T), np.argmax(inp.T), np.argmin(inp.eta_e), np.argmax(inp.eta_e)):
        take([int(c)], 1)
    corner = np.nonzero((inp.eta_e > 30.0) & (inp.T < 2.0))[0]
    take(corner, int(round(corner_share * count)))
    lt = np.log(inp.T)
    tb = np.minimum(((lt - lt.min()) / max(lt.max() - lt.min(), 1e-300) * cells).astype(np.int64), cells - 1)
    eb = np.minimum(((inp.eta_e - inp.eta_e.min()) / max(inp.eta_e.max() - inp.eta_e.min(), 1e-300) * cells)
                    .astype(np.int64), cells - 1)
    cell = tb * cells + eb
    order = np.argsort(cell, kind="stable")
    bounds = np.searchsorted(cell[order], np.arange(cells * cells + 1))
    left = count - len(chosen)
    for c in range(cells * cells):
        share = left // (cells * cells - c)
        before = len(chosen)
        take(order[bounds[c]:bounds[c + 1]], share)
        left -= len(chosen) - before
    if left > 0:
        take(np.arange(nz), left)
    return np.array(sorted(chosen[:count]), dtype=np.int64)


GRAD_PERIOD = 4099


def gradient_pool(ne: int, seed: int, period: int = GRAD_PERIOD):
    """Seeded upstream-gradient rows g_eta, g_chi [period, 3, 2, NE] (unit normals). Zone z of a
    workload takes row z mod period, so a full-size workload's gradients are a gather on any
    device and the rows of sampled zones are known without drawing the rest."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 2500 + seed))
    return (rng.standard_normal((period, NSPECIES, 2, ne)), rng.standard_normal((period, NSPECIES, 2, ne)))


def pooled_gradients(idx, ne: int, seed: int, period: int = GRAD_PERIOD):
    """The pool rows of the zones idx (see gradient_pool)."""
    ge, gc = gradient_pool(ne, seed, period)
    r = np.asarray(idx) % period
    return np.ascontiguousarray(ge[r]), np.ascontiguousarray(gc[r])
