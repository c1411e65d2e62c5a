"""bench.py's JSON line on the GPU: a short run of the 512^2 x 720 x 725 solve
(with the CPU oracle leg) prints one line with every field of the contract,
consistent with itself: value = steps / timed seconds, roofline.frac =
achieved / peak, the roofline kernel among the two projector kernels, and a
CPU baseline from the oracle."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_line_contract():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("bench --steps 5 (contract)", flush=True)
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "5", "--warmup", "1", "--reps", "3",
           "--no-batch", "--no-learned", "--no-quality", "--no-stored", "--no-large"]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stderr[-3000:]
    lines = [ln for ln in res.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, res.stdout[-2000:]
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 5 and d["warmup"] == 1
    assert d["unit"] == "iterations/s" and d["higher_is_better"] is True
    assert d["value"] > 0 and abs(d["ms_per_step"] - 1000.0 / d["value"]) <= 1e-3 * d["ms_per_step"] + 1e-3
    assert isinstance(d["config"]["workload"], str) and "512x512" in d["config"]["workload"]
    r = d["roofline"]
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in r, key
    assert r["bound"] in ("hbm", "mfma", "alu")
    assert r["kernel"] in ("project", "backproject")
    assert abs(r["frac"] - r["achieved"] / r["peak"]) <= 1e-3 and 0.0 < r["frac"] <= 1.0
    for name in ("project", "backproject"):
        k = r["kernels"][name]
        assert k["ms"] > 0 and 0.0 < k["frac"] <= 1.0 and 0.0 < k["valu_issue"]["frac"] <= 1.0
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["value"] > 0 and c["cores"] >= 1
    assert c["unit"] == d["unit"] and isinstance(c["sample"], str)
