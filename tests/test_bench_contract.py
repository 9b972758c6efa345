"""The bench's command-line contract.

  * CPU: more than one GPU is refused with a message and exit status 2,
    before anything touches a GPU;
  * GPU: one short run on the smallest workload prints one JSON line with the
    fields the contract names (metric, value, unit, ..., roofline), and the
    figures agree with each other: value x ms_per_step = N particle-steps,
    roofline.frac = achieved / peak, the modes' drift and footprint present.
"""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""


@pytest.mark.gpu
def test_short_run_prints_the_contract_line():
    print("[bench contract] lj4k, 20 steps", flush=True)
    p = subprocess.run([sys.executable, "-u", BENCH, "--config", "lj4k", "--steps", "20", "--warmup", "2",
                        "--no-cpu", "--protocol-steps", "0"], capture_output=True, text=True, timeout=240)
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [ln for ln in p.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    j = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in j, key
    assert j["n_gpus"] == 1 and j["steps"] == 20 and j["warmup"] == 2
    assert j["higher_is_better"] is True and j["scaling"] == "weak"
    assert j["cpu_baseline"] is None   # --no-cpu
    assert isinstance(j["config"]["workload"], str) and j["config"]["workload"].startswith("lj4k")
    n = j["config"]["n"]
    assert j["value"] > 0 and j["ms_per_step"] > 0
    assert j["value"] * j["ms_per_step"] * 1e-3 == pytest.approx(n, rel=1e-9)
    r = j["roofline"]
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in r, key
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], abs=1e-4)   # both printed rounded
    modes = j["modes"]
    assert set(modes) == {"fp64"}   # lj4k runs FP64 alone
    m = modes["fp64"]
    assert m["hbm_footprint_bytes"] > 0 and m["list_cell_stride_end"] >= m["list_cell_stride"]
    assert m["rebuilds"] >= 1 and m["force_kernel"]["launches"] == 20
