"""Register budget of the compiled kernels (host only: hipcc cross-compiles gfx950 to ISA).

The kernels are bound by VALU instruction issue, so their speed rests on the occupancy each
was designed for: waves per SIMD set by VGPRs (512 per lane, allocated in blocks of 8) and
by LDS. A change that makes a kernel spill to scratch, or grow past the VGPRs of its
occupancy target, costs time without failing any numerical test. This test compiles the
device code with the library's own flags and reads the code-object metadata:

* no kernel uses scratch (private segment) or spills VGPRs;
* the FP32 forward and interpolation kernels fit five waves per SIMD (at most 96 VGPRs);
* the FP32 backward and the FP64 forward fit three (at most 168);
* the FP64 backward and the FP64 export of task values for tables fit two (at most 256);
* the forward with the electron mass (FP64, one 256-lane workgroup per zone) fits two;
* the ray solve (a 1024-lane workgroup per ray, four waves per SIMD) fits in 128.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_1404_1719_amd import build_lib

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# kernel-name pattern -> the most VGPRs its waves-per-SIMD target allows
BUDGET = [
    (r"rates_forward_kernelINS0_4Fp32", 96),
    (r"rates_interp_kernel", 96),
    (r"rates_backward_kernelINS0_4Fp32", 168),
    (r"rates_forward_kernelINS0_4Fp64ELi[01]E", 168),
    (r"rates_forward_kernelINS0_4Fp64ELi[23]E", 256),
    (r"rates_backward_kernelINS0_4Fp64", 256),
    (r"rates_mass_kernel", 256),
    (r"ray_solve_kernel", 128),
]


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    flags = [f for f in build_lib.FLAGS if f not in ("-shared", "-fPIC")]
    text = ""
    for name in ("vtx_kernels", "vtx_massive", "vtx_newton"):
        out = tmp_path_factory.mktemp("isa") / (name + ".s")
        src = os.path.join(build_lib.CSRC, name + ".hip")
        subprocess.run([HIPCC] + flags + ["--cuda-device-only", "-S", "-o", str(out), src], check=True,
                       capture_output=True)
        text += out.read_text()
    meta = {}
    for blk in text.split("  - .agpr_count")[1:]:
        name = re.search(r"\.name:\s+(\S+)", blk).group(1)

        def field(key):
            m = re.search(r"\." + key + r":\s+(\d+)", blk)
            return int(m.group(1)) if m else None

        meta[name] = {"vgpr": field("vgpr_count"), "scratch": field("private_segment_fixed_size"),
                      "vspill": field("vgpr_spill_count")}
    assert meta, "no kernel metadata found"
    return meta


def test_no_kernel_uses_scratch(kernels):
    for name, m in kernels.items():
        assert m["scratch"] == 0, (name, m)
        assert not m["vspill"], (name, m)


def test_vgprs_fit_the_occupancy_targets(kernels):
    seen = set()
    for name, m in kernels.items():
        for pat, cap in BUDGET:
            if re.search(pat, name):
                assert m["vgpr"] <= cap, (name, m["vgpr"], cap)
                seen.add(pat)
                break
    assert seen == {p for p, _ in BUDGET}, seen
