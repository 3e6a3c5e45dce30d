"""The benchmark script's contract: one GPU only (a clear refusal for more),
the committed HBM-traffic record is picked up only for the exact kernel
source and tilings it was measured with, and (on a GPU) one JSON line with
the required keys."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def _record():
    rec = {}
    for line in open(os.path.join(ROOT, "profiles", "k_mttkrp_f64_c2_traffic.md")):
        if ":" in line and not line.startswith(("#", " ", "|")):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    return rec


def test_traffic_record_matches_only_its_tilings():
    rec = _record()
    tilings = [t.strip() for t in rec["tiling"].split(";")]
    assert bench.measured_traffic("c2", "fp64", tilings) == int(rec["traffic_bytes_per_launch"])
    assert bench.measured_traffic("c2", "fp64", tilings[:-1]) is None
    assert bench.measured_traffic("c2", "bf16x3", tilings) is None
    assert bench.measured_traffic("c3", "fp64", tilings) is None


@pytest.mark.gpu
def test_bench_prints_one_json_line():
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--steps", "1",
                        "--warmup", "0", "--sweeps", "12", "--no-cpu", "--no-plain"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["value"] > 0 and d["dtype"] == "f64"
    assert "workload" in d["config"]
    roof = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in roof, k
    assert 0 < roof["frac"] < 1 and roof["peak"] == 78.6


def test_shipped_tuning_table_covers_every_benchmark_workload():
    """The tuned tilings bench.py times, and the full-size tests force, exist
    for every workload: each mode, plus W for 3-way float64 problems.  The
    shapes are those of the synthetic workloads (100x200x200 with 100 rank-5
    models; 300x250x200 with ranks 1..10 x 5 inits x 300 samples; the 4-way
    200x120x100x80 with 200 rank-12 models in both splits; 100x150x150
    float32 with 100 rank-10 models)."""
    from types import SimpleNamespace

    import numpy as np

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gpu_util import shipped_tilings

    def wl(dims, C, dtype=np.float64):
        return SimpleNamespace(dims=dims, ranks=np.array([C]), T=np.empty(0, dtype))

    cases = [(wl((100, 200, 200), 500), 0, 4), (wl((300, 250, 200), 82500), 0, 4),
             (wl((100, 150, 150), 1000, np.float32), 0, 4),
             (wl((200, 120, 100, 80), 2400), 1, 4), (wl((200, 120, 100, 80), 2400), 2, 4)]
    for w, precision, slots in cases:
        t = shipped_tilings(w, precision)
        assert sorted(t) == list(range(slots)), (w.dims, precision, sorted(t))
        for geo, splits in t.values():
            assert len(geo) == 6 and splits >= 1
