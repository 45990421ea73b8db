"""Pins for the tabulated-kernel oracle (oracle.tabulated)."""
import numpy as np

from oracle import rates, tabulated
from paper_1404_1719_amd import synth


def test_layout_round_trip():
    inp = synth.make_inputs("medium", nzones=3)
    for proc in (3, 7, 1, 2, 4):
        opts = rates.Options(nquad=32, processes=proc)
        quad = rates.task_quadratures(inp.eps, inp.T, inp.eta_e, opts)
        vec = tabulated.pack(quad, len(inp.eps))
        assert vec.shape == (3, tabulated.values_per_zone(len(inp.eps), opts))
        back = tabulated.unpack(vec, len(inp.eps), opts)
        for k in quad:
            assert np.array_equal(back[k], quad[k])
        direct = rates.zone_kernels(inp.eps, inp.T, inp.eta_e, opts)
        again = rates.complete(inp.eps, inp.T, back)
        for k in direct:
            assert np.array_equal(direct[k], again[k])


def test_nodes_reproduce_the_direct_rates():
    inp = synth.make_inputs("medium", nzones=4)
    lat = tabulated.Lattice(nt=3, nh=4, lnT0=np.log(2.0), dlnT=0.5, eta0=1.0, deta=3.0)
    opts = rates.Options(nquad=32)
    table = tabulated.build(inp.eps, lat, opts)
    T, eta = tabulated.lattice_states(lat)
    f = np.repeat(inp.f[:1], T.shape[0], axis=0)
    e1, c1 = tabulated.forward(inp.eps, inp.w, lat, table, T, eta, f, opts)
    e0, c0, ae, ac = rates.forward_with_scale(inp.eps, inp.w, T, eta, f, opts)
    assert np.all(np.abs(e1 - e0) <= 1e-12 * ae) and np.all(np.abs(c1 - c0) <= 1e-12 * ac)


def test_exact_on_bilinear_data():
    """Data bilinear in the lattice coordinates are reproduced exactly by ``bilinear``; pairs
    with ln x0 and x1/x0 bilinear (exponential dependence) exactly by ``interpolate``."""
    lat = tabulated.Lattice(nt=5, nh=7, lnT0=-0.5, dlnT=0.3, eta0=-2.0, deta=1.5)
    rng = np.random.default_rng(3)
    al, be, ga, de = rng.normal(size=(4, 10))
    a, b = np.meshgrid(np.arange(lat.nt), np.arange(lat.nh), indexing="ij")
    s, r = a.ravel()[:, None], b.ravel()[:, None]
    lin = al + be * s + ga * r + de * s * r
    T = np.exp(rng.uniform(-1.5, 2.0, 50))          # inside and outside the lattice
    eta = rng.uniform(-5.0, 12.0, 50)
    s = ((np.log(T) - lat.lnT0) / lat.dlnT)[:, None]
    r = ((eta - lat.eta0) / lat.deta)[:, None]
    ref = al + be * s + ga * r + de * s * r
    assert np.allclose(tabulated.bilinear(lin, lat, T, eta), ref, rtol=1e-12, atol=1e-12)
    raw = np.empty_like(lin)
    raw[:, 0::2] = np.exp(lin[:, 0::2])
    raw[:, 1::2] = lin[:, 1::2] * raw[:, 0::2]
    table = tabulated.to_interp_vars(raw)
    assert np.allclose(table, lin, rtol=1e-12, atol=1e-12)
    got = tabulated.interpolate(table, lat, T, eta)
    x0 = np.exp(ref[:, 0::2])
    assert np.allclose(got[:, 0::2], x0, rtol=1e-12, atol=0)
    assert np.allclose(got[:, 1::2], ref[:, 1::2] * x0, rtol=1e-12, atol=1e-300)


def test_second_order_convergence():
    """Halving the lattice spacing cuts the interpolation error of eta0 about fourfold (zone
    states whose cells hold no breakpoint crossing of the rule)."""
    inp = synth.make_inputs("medium", nzones=1)
    opts = rates.Options(nquad=32)
    T, eta = np.array([7.3]), np.array([3.1])
    f = inp.f[:1]
    e0, c0 = rates.forward(inp.eps, inp.w, T, eta, f, opts)
    errs = []
    for h in (0.2, 0.1, 0.05):
        lat = tabulated.Lattice(nt=3, nh=3, lnT0=np.log(7.3) - 1.3 * h, dlnT=h, eta0=3.1 - 0.6 * h, deta=h)
        table = tabulated.build(inp.eps, lat, opts)
        e1, _ = tabulated.forward(inp.eps, inp.w, lat, table, T, eta, f, opts)
        errs.append(np.max(np.abs(e1 - e0)[:, :, 0] / np.abs(e0[:, :, 0])))
    assert errs[1] < 0.35 * errs[0] and errs[2] < 0.35 * errs[1], errs
