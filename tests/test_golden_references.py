"""The stored oracle references of the full-size GPU parity tests and of the benchmark's error
report (tests/golden/ref_<workload>.npz, written by tests/golden/make_reference.py).

* They were written from the current oracle and sampler: the stored source hash matches.
* Their layout is whole: a stratified sample with the extreme zones and the corner
  eta_e > 30, T < 2 MeV, a backward sub-sample inside it, finite values.
* For the medium workload (cheap to draw) the sample is the sampler's, the stored zone states
  are the workload's, and the oracle recomputed on a few stored zones gives the stored values
  bit for bit (the float32 gradient scale to its rounding).
* The gradient scale aq_g_f bounds |g_f| (it sums the absolute values of g_f's terms).
"""
import os
import sys

import numpy as np
import pytest

from paper_1404_1719_amd import synth

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_reference  # noqa: E402


@pytest.mark.parametrize("name", sorted(make_reference.PLAN))
def test_reference_is_current_and_whole(name):
    ref = make_reference.load(name)
    assert str(ref["source_hash"]) == make_reference.source_hash(), "oracle changed: rerun make_reference.py"
    nf, nb = make_reference.PLAN[name]
    ne = synth.WORKLOADS[name].ne
    idx, idx_b = ref["idx"], ref["idx_b"]
    assert idx.shape == (nf,) and idx_b.shape == (nb,)
    assert np.all(np.diff(idx) > 0) and np.all(np.isin(idx_b, idx))
    assert ref["eta"].shape == (nf, 3, 2, ne) and ref["g_f"].shape == (nb, 3, 2, ne)
    for k in ("eta", "chi", "a_eta", "a_chi", "aq_eta", "aq_chi", "g_T", "g_eta_e", "g_f", "aq_g_f"):
        assert np.all(np.isfinite(ref[k])), k
    # the gradient's absolute scale bounds it: |J^T g| <= |J|_abs^T |g|
    assert ref["aq_g_f"].shape == ref["g_f"].shape
    assert np.all(ref["aq_g_f"].astype(np.float64) >= np.abs(ref["g_f"]) * (1 - 1e-6))
    # |integral of H B| <= integral of |H| B: the quadrature-level scale bounds the output level
    for o in ("eta", "chi"):
        a, aq = ref["a_" + o].astype(np.float64), ref["aq_" + o].astype(np.float64)
        assert np.all(aq >= a * (1 - 1e-6)), o
        assert np.allclose(aq[:, :, 0], a[:, :, 0], rtol=1e-6, atol=0), o   # l = 0: H >= 0
    if "T" in ref:
        T, E = ref["T"], ref["eta_e"]
        assert np.sum((E > 30) & (T < 2)) >= (nf // 10 if name == "large" else 1)


def test_electron_mass_reference_is_current_and_whole():
    ref = make_reference.load("lowt")
    assert str(ref["source_hash"]) == make_reference.source_hash(("oracle/massive.py",))
    n = make_reference.PLAN_MASS["lowt"]
    assert ref["idx"].shape == (n,) and np.all(np.diff(ref["idx"]) > 0)
    assert ref["eta"].shape == (n, 3, 2, synth.WORKLOADS["lowt"].ne)
    for k in ("eta", "chi", "a_eta", "a_chi"):
        assert np.all(np.isfinite(ref[k])), k
    inp = synth.make_inputs("lowt")
    assert np.array_equal(synth.sample_zones_stratified(inp, n, make_reference.SAMPLE_SEED), ref["idx"])
    assert np.array_equal(inp.T[ref["idx"]], ref["T"])


def test_medium_reference_reproduces():
    from oracle import grad as ograd
    from oracle import rates as orates
    ref = make_reference.load("medium")
    wl = synth.WORKLOADS["medium"]
    inp = synth.make_inputs("medium")
    idx, idx_b = make_reference.samples(inp, *make_reference.PLAN["medium"])
    assert np.array_equal(idx, ref["idx"]) and np.array_equal(idx_b, ref["idx_b"])
    assert np.array_equal(inp.T[idx], ref["T"]) and np.array_equal(inp.eta_e[idx], ref["eta_e"])
    opts = orates.Options(nquad=wl.nquad, rule=wl.rule)
    pos = [0, 500, len(idx) - 1]
    sub = synth.subset(inp, idx[pos])
    e, c, _, _ = orates.forward_with_scale(sub.eps, sub.w, sub.T, sub.eta_e, sub.f, opts)
    assert np.allclose(e, ref["eta"][pos], rtol=1e-14, atol=0) and np.allclose(c, ref["chi"][pos], rtol=1e-14, atol=0)
    zb = [3]
    sb = synth.subset(inp, idx_b[zb])
    ge, gc = synth.pooled_gradients(idx_b[zb], wl.ne, int(ref["grad_seed"]))
    gT, gE, gf = ograd.vjp(sb.eps, sb.w, sb.T, sb.eta_e, sb.f, ge, gc, opts)
    assert np.allclose(gT, ref["g_T"][zb], rtol=1e-13, atol=0) and np.allclose(gf, ref["g_f"][zb], rtol=1e-12,
                                                                                  atol=1e-300)
    J = orates.jacobian(sb.eps, sb.w, sb.T, sb.eta_e, opts, absolute=True)
    assert np.allclose(make_reference.grad_f_scale(J, ge, gc), ref["aq_g_f"][zb], rtol=1e-6, atol=0)
