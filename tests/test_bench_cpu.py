"""Host-side checks of bench.py: the multi-GPU refusal and the CPU-baseline leg (the
FP64 oracle on a tiny workload), so that the benchmark's own code paths are exercised
without a GPU."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_cpu_baseline_leg_runs_the_oracle():
    sys.path.insert(0, ROOT)
    import bench
    from synth import make_config
    d = make_config("slice64_c4_t16_k3")
    cfg = dict(d["cfg"])
    out = bench.cpu_baseline(d["classes"][0], d["phi"], cfg, 1, 1)
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["unit"] == "slices/s"
    assert out["value"] > 0 and "1 of 20" in out["sample"]


def test_workloads_are_looked_up_by_name():
    sys.path.insert(0, ROOT)
    import pytest
    from synth import CONFIGS, make_config
    assert all(k == v["name"] for k, v in CONFIGS.items())
    for bad in (4, "vol512", ""):
        with pytest.raises(KeyError):
            make_config(bad)
