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


def test_committed_bench_line_is_self_consistent():
    """The committed bench line's derived figures follow from its own measurements:
    achieved bandwidth = algorithmic bytes per launch / average launch time, frac =
    achieved / peak, slices/s = slices / seconds per volume; its traffic fields are
    the counter summary's figures for the same kernel; and the kernel-trace summary
    of the same workload gives the dominant kernel's average launch time within 2 %."""
    prof = os.path.join(ROOT, "profiles")
    b = json.load(open(os.path.join(prof, "bench_vol512_384x384_c16_t100_k5.json")))
    r = b["roofline"]
    assert abs(r["achieved"] - r["alg_bytes_per_launch"] / r["avg_launch_ms"] / 1e6) < 1e-3 * r["achieved"]
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    assert b["kernels"][r["kernel"]]["avg_ms"] == r["avg_launch_ms"]
    assert abs(b["value"] - b["slices_completed"] / b["s_per_volume"]) < 1e-2
    t = json.load(open(os.path.join(prof, "hbm_traffic_vol512_384x384_c16_t100_k5.json")))
    tk = t["traffic"][r["kernel"]]
    assert t["workload"] == b["config"]["workload"]
    assert abs(r["traffic"] - tk["bytes_per_launch"]) <= 1
    assert abs(r["traffic_vs_alg"] - tk["ratio_to_alg"]) < 1e-3
    rows = [ln for ln in open(os.path.join(prof, "kernel_stats_vol512_384x384_c16_t100_k5.md"))
            if ln.startswith("| `") and "k_passB<384, 5>" in ln]
    assert len(rows) == 1
    avg_ms = int(rows[0].split("|")[4]) / 1e6
    assert abs(avg_ms - r["avg_launch_ms"]) < 0.02 * r["avg_launch_ms"]
