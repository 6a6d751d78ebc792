"""bench.py's output line on the GPU: one JSON line with the fields the benchmark contract names
(metric, value, unit, n_gpus, steps, warmup, ms_per_step, higher_is_better, scaling, vs_baseline,
dtype, data, config with a workload, roofline with bound / achieved / peak / unit / frac /
traffic), run in this process on the small 1D shock with a few steps."""
import json
import os
import sys

import pytest

from tests.gpu_util import HAVE_GPU, banner, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bench_line_has_the_contract_fields(capsys):
    import bench
    banner("bench.py --workload shock1d --steps 4 --warmup 2 --no-extras --no-cpu-baseline")
    assert bench.main(["--workload", "shock1d", "--steps", "4", "--warmup", "2", "--no-extras",
                       "--no-cpu-baseline"]) == 0
    lines = [l for l in capsys.readouterr().out.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 4 and d["warmup"] == 2 and d["higher_is_better"] is True
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["dtype"] == "f32" and d["data"] == "synthetic"
    assert "workload" in d["config"] and "model" not in d["config"]
    r = d["roofline"]
    assert r["bound"] in ("hbm", "mfma", "alu") and r["unit"] in ("GB/s", "TFLOP/s")
    assert 0 < r["achieved"] and 0 < r["frac"] < 1 and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-9
    assert "traffic" in r
    assert d["tuning"]["cells_per_block"] in (16, 32, 64, 128, 256)
