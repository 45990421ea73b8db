"""Tabulated kernels with interpolation (oracle; test infrastructure only).

A production alternative to evaluating the kernel quadratures for every zone: evaluate them
once on a regular lattice of zone states in (ln T, eta_e), then interpolate them for each
zone, and complete and contract as usual. Detailed-balance and production factors take
the zone's own T, so detailed balance stays exact; the interpolation error sits in the
quadratures alone. The paper evaluates the rates per zone (Sect. 2.1 lists them as a model
component); this is a comparison point, not the paper's method.

Export layout of one zone's quadratures (the order in which the library writes them):
  scattering q[t][S][l] (4 ntn values, tasks t = (i >= j) in ``rates.nes_tasks`` order),
  scattering on positrons likewise (4 ntn, when PROC_NPS), pair A[i][j][l] (2 ne^2).
Lattice: node (a, b), a < nt, b < nh, at ln T = lnT0 + a dlnT, eta_e = eta0 + b deta; its
row in the table is a nh + b.
Interpolation variables: the layout holds each (task, S) as the pair (l = 0, l = 1), adjacent.
Phi_0 is positive and varies exponentially with 1/T and eta_e; |Phi_1| <= Phi_0 because
|P_1| <= 1 under a nonnegative rate. The table stores a pair (x0, x1) as (ln x0, x1/x0) (x0 <= 0,
only from underflow, as (ln 1e-300, 0)); interpolated rows map back by x0 = exp(y0), x1 = y1 x0.
Interpolation: bilinear in s = (ln T - lnT0)/dlnT and r = (eta_e - eta0)/deta on the cell
a = clip(floor(s), 0, nt - 2), b = clip(floor(r), 0, nh - 2), with u = s - a, v = r - b
(outside the lattice this extrapolates linearly from the edge cell).

Pins: tests/test_oracle_tabulated.py (layout round trip, node values, exactness on bilinear
data, second-order convergence).
"""
import dataclasses

import numpy as np

from . import rates


@dataclasses.dataclass(frozen=True)
class Lattice:
    nt: int
    nh: int
    lnT0: float
    dlnT: float
    eta0: float
    deta: float


def values_per_zone(ne, opts):
    ntn = ne * (ne + 1) // 2
    n = 0
    if opts.processes & rates.PROC_NES:
        n += 4 * ntn
    if opts.processes & rates.PROC_NPS:
        n += 4 * ntn
    if opts.processes & rates.PROC_PAIR:
        n += 2 * ne * ne
    return n


def pack(quad, ne):
    """[z, values] in the export layout from the dict of ``rates.task_quadratures``."""
    parts = []
    for name in ("nes", "nps"):
        if name in quad:
            q = quad[name]
            parts.append(q.reshape(q.shape[0], -1))      # [z, t, S, l] -> t-major
    if "pair" in quad:
        A = quad["pair"]
        parts.append(A.reshape(A.shape[0], -1))          # [z, i, j, l]
    return np.concatenate(parts, axis=1)


def unpack(vec, ne, opts):
    ntn = ne * (ne + 1) // 2
    out, off = {}, 0
    nz = vec.shape[0]
    for bit, name in ((rates.PROC_NES, "nes"), (rates.PROC_NPS, "nps")):
        if opts.processes & bit:
            out[name] = vec[:, off:off + 4 * ntn].reshape(nz, ntn, 2, 2)
            off += 4 * ntn
    if opts.processes & rates.PROC_PAIR:
        out["pair"] = vec[:, off:off + 2 * ne * ne].reshape(nz, ne, ne, 2)
        off += 2 * ne * ne
    assert off == vec.shape[1]
    return out


def lattice_states(lat):
    """(T, eta_e) of the lattice nodes in table-row order."""
    a, b = np.meshgrid(np.arange(lat.nt), np.arange(lat.nh), indexing="ij")
    return np.exp(lat.lnT0 + a.ravel() * lat.dlnT), lat.eta0 + b.ravel() * lat.deta


def build(eps, lat, opts, chunk=32):
    """The table [nt nh, values]: the quadratures at every lattice node, in interpolation
    variables."""
    T, eta = lattice_states(lat)
    rows = [pack(rates.task_quadratures(eps, T[k:k + chunk], eta[k:k + chunk], opts), len(eps))
            for k in range(0, T.shape[0], chunk)]
    return to_interp_vars(np.concatenate(rows))


def to_interp_vars(x):
    """(x0, x1) pairs -> (ln x0, x1 / x0)."""
    x0, x1 = x[..., 0::2], x[..., 1::2]
    pos = x0 > 0
    y = np.empty_like(x)
    y[..., 0::2] = np.log(np.where(pos, x0, 1e-300))
    y[..., 1::2] = np.where(pos, x1 / np.where(pos, x0, 1.0), 0.0)
    return y


def from_interp_vars(y):
    x = np.empty_like(y)
    x0 = np.exp(y[..., 0::2])
    x[..., 0::2] = x0
    x[..., 1::2] = y[..., 1::2] * x0
    return x


def bilinear(table, lat, T, eta_e):
    """Bilinear interpolation of the table rows at zone states (T, eta_e): [z, values]."""
    s = (np.log(np.asarray(T, dtype=float)) - lat.lnT0) / lat.dlnT
    r = (np.asarray(eta_e, dtype=float) - lat.eta0) / lat.deta
    a = np.clip(np.floor(s), 0, lat.nt - 2).astype(int)
    b = np.clip(np.floor(r), 0, lat.nh - 2).astype(int)
    u = (s - a)[:, None]
    v = (r - b)[:, None]
    t00 = table[a * lat.nh + b]
    t10 = table[(a + 1) * lat.nh + b]
    t01 = table[a * lat.nh + b + 1]
    t11 = table[(a + 1) * lat.nh + b + 1]
    return (1 - u) * (1 - v) * t00 + u * (1 - v) * t10 + (1 - u) * v * t01 + u * v * t11


def interpolate(table, lat, T, eta_e):
    """Task values at zone states (T, eta_e) from a table in interpolation variables."""
    return from_interp_vars(bilinear(table, lat, T, eta_e))


def forward(eps, w, lat, table, T, eta_e, f, opts=rates.Options()):
    """eta, chi from interpolated quadratures, completed and contracted with the zones' own T."""
    T = np.asarray(T, dtype=float)
    quad = unpack(interpolate(table, lat, T, eta_e), len(eps), opts)
    return rates.contract(rates.complete(eps, T, quad), w, f, opts)
