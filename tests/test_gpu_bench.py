"""The benchmark's output contract (needs a gfx950 GPU): bench.py, run as a separate process on
the small workload, prints exactly one JSON line with the metric, the whole-job value and its
configuration, the roofline of the dominant call and the CPU-oracle baseline, and its value is
the zone*(eps, eps') pairs of one step over the measured step time."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KEYS = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
        "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline")


def test_bench_line_small_workload():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "small", "--steps", "3", "--warmup", "1"]
    print("[gpu] " + " ".join(cmd[1:]), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=280, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, r.stdout[-2000:]
    d = json.loads(lines[0])
    for k in KEYS:
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1
    assert d["higher_is_better"] is True and d["data"] == "synthetic" and d["vs_baseline"] is None
    cfg = d["config"]
    assert cfg["workload"].startswith("small")   # the small workload is plain FP64
    assert (cfg["precision"], d["dtype"]) in (("fp64", "f64"), ("mixed", "f32+f64"))
    pairs = cfg["zones"] * cfg["ne"] ** 2
    assert d["value"] > 0 and d["ms_per_step"] > 0
    assert abs(d["value"] * d["ms_per_step"] * 1e-3 / pairs - 1.0) < 1e-6
    ro = d["roofline"]
    assert ro["bound"] in ("hbm", "mfma", "alu") and ro["unit"] in ("GB/s", "TFLOP/s")
    assert ro["achieved"] > 0 and ro["peak"] > 0 and abs(ro["frac"] - ro["achieved"] / ro["peak"]) < 1e-9
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1 and cb["sample"]
    print(f"    value {d['value']:.3e} {d['unit']}, roofline frac {ro['frac']:.3f}, "
          f"oracle {cb['value']:.3e} on {cb['cores']} cores", flush=True)
