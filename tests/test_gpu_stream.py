"""GPU test of the chunked host-memory streaming driver (paper_1404_1719_amd.stream).

The medium workload (102,400 zones) in pinned host memory, 8 chunks: inputs by DMA on a copy
stream, forward and backward of each chunk on two compute streams, outputs written into the
mapped host arrays. Its outputs equal, bit for bit, those of the same calls on device-resident
inputs, and match the stored FP64 oracle reference (tests/golden/ref_medium.npz) on its
sampled zones within the bars (FP64 1e-6 against the output-level floor, mixed 1e-4 against the
quadrature-level one, as in test_gpu_scale).
"""
import os
import sys

import numpy as np
import pytest

from paper_1404_1719_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1404_1719_amd import stream, vtx  # noqa: E402

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_reference  # noqa: E402

DEV = "cuda:0"
TOL = {"fp64": 1e-6, "mixed": 1e-4}


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_streamed_equals_resident_and_oracle(precision):
    name = "medium"
    wl = synth.WORKLOADS[name]
    inp = synth.make_inputs(name)
    ref = make_reference.load(name)
    nz = inp.T.shape[0]
    pe, pc = synth.gradient_pool(wl.ne, int(ref["grad_seed"]))
    rows = np.arange(nz) % pe.shape[0]
    ge, gc = pe[rows], pc[rows]
    grid = vtx.GridHandle(inp.eps, inp.w)
    opts = vtx.make_opts(precision, wl.nquad, wl.rule)
    print(f"[gpu] streaming {name} {precision}: {nz} zones in 8 chunks", flush=True)
    st = stream.Streamer(grid, opts, nz, chunks=8)
    for k, v in (("T", inp.T), ("eta_e", inp.eta_e), ("f", inp.f), ("g_eta", ge), ("g_chi", gc)):
        st.host[k].copy_(torch.from_numpy(np.ascontiguousarray(v)))
    st.step()
    st.synchronize()
    # the same calls on device-resident inputs, same chunks
    d = {k: torch.from_numpy(np.ascontiguousarray(v)).to(DEV)
         for k, v in (("T", inp.T), ("E", inp.eta_e), ("f", inp.f), ("ge", ge), ("gc", gc))}
    eta, chi = torch.empty_like(d["f"]), torch.empty_like(d["f"])
    gT, gE, gf = torch.empty_like(d["T"]), torch.empty_like(d["T"]), torch.empty_like(d["f"])
    for a, b in st.chunks:
        vtx.forward(grid, opts, d["T"][a:b], d["E"][a:b], d["f"][a:b], eta[a:b], chi[a:b])
        vtx.backward(grid, opts, d["T"][a:b], d["E"][a:b], d["f"][a:b], d["ge"][a:b], d["gc"][a:b], gT[a:b],
                     gE[a:b], gf[a:b])
    torch.cuda.synchronize()
    for k, t in (("eta", eta), ("chi", chi), ("g_T", gT), ("g_eta_e", gE), ("g_f", gf)):
        assert torch.equal(st.host[k], t.cpu()), k
    idx, idx_b = ref["idx"], ref["idx_b"]
    H = {k: st.host[k].numpy() for k in ("eta", "chi", "g_T", "g_eta_e", "g_f")}

    def ferr(y, r, a):
        return np.max(np.abs(y - r) / np.maximum(np.maximum(np.abs(r), fl * a.astype(np.float64)), 1e-290))

    def gerr(g, r):
        return np.max(np.abs(g - r) / np.maximum(np.abs(r), 1e-3 * np.mean(np.abs(r)) + 1e-300))

    # floors as in the full-size parity tests: mixed 1e-2 Aq (FP32 rounding of the quadrature
    # over |H|), FP64 1e-3 A
    sc, fl = ("aq", 1e-2) if precision == "mixed" else ("a", 1e-3)
    e = max(ferr(H["eta"][idx], ref["eta"], ref[sc + "_eta"]), ferr(H["chi"][idx], ref["chi"], ref[sc + "_chi"]))
    g = max(gerr(H[k][idx_b], ref[k]) for k in ("g_T", "g_eta_e"))
    g = max(g, ferr(H["g_f"][idx_b], ref["g_f"], ref["aq_g_f"]) if precision == "mixed"
            else gerr(H["g_f"][idx_b], ref["g_f"]))
    print(f"    bit-equal to the resident calls; vs oracle: forward {e:.2e} ({idx.size} zones), "
          f"backward {g:.2e} ({idx_b.size} zones)", flush=True)
    assert e <= TOL[precision] and g <= TOL[precision]
