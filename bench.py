"""Throughput of the T2-Shuffling slice reconstruction on one MI355X.

Workload (default): the 320-slice 256 x 256 volume, C = 8 coils, T = 80 echoes,
K = 4, 1.5 % VD Poisson-disc sampling per echo, 8 x 8 LLR blocks, lambda = 0.01,
rho = 0.1, 100 ADMM outer x 5 CG iterations, synthetic (seeded) data.

One step = the whole hot path over the volume: projection + adjoint of the
device-resident samples (t2s_load_slices) and the full ADMM solve
(t2s_reconstruct), all slices batched per launch.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "readout slices/s & s/volume at equal ADMM residual: plain vs batched+warm-start"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on the host cores, one slice per process
# ---------------------------------------------------------------------------

_CPU = {}


def _oracle_job(i):
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import t2s as O
    d = _CPU
    t0 = time.perf_counter()
    O.admm(d["ksp"][i], d["sens"][i], d["phi"], d["masks"], d["lam"], d["rho"], d["block"], d["outer"], d["n_cg"],
           d["seed"], g=int(d["g"][i]))
    return time.perf_counter() - t0


def cpu_baseline(cl, phi, cfg, n_procs, outer):
    """Run the oracle on n_procs slices for `outer` outer iterations each, in parallel."""
    sel = np.linspace(0, cl.nslices - 1, n_procs).round().astype(int)
    _CPU.update(ksp=cl.ksp[sel], sens=cl.sens[sel], phi=phi, masks=cl.masks.astype(bool), lam=cfg["lam"],
                rho=cfg["rho"], block=cfg["block"], outer=outer, n_cg=cfg["n_cg"], seed=cfg["seed"], g=sel)
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(n_procs) as pool:
        per = pool.map(_oracle_job, range(n_procs))
    wall = time.perf_counter() - t0
    # full-schedule slices completed per second
    frac = outer / cfg["n_outer"]
    return dict(value=n_procs * frac / wall, unit="slices/s", cores=n_procs, kind="oracle",
                sample=f"{n_procs} slices x {outer} of {cfg['n_outer']} ADMM outer iterations (5 CG), FP64 NumPy, "
                       f"one process per slice, wall {wall:.1f} s, per-slice {np.mean(per):.1f} s",
                s_per_volume=cl.nslices / (n_procs * frac / wall))


# ---------------------------------------------------------------------------


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=1, help="workload id (1: 320 x 256^2 volume)")
    ap.add_argument("--mode", choices=["batched", "graph", "per_slice"], default="batched",
                    help="launch schedule; 'graph' replays a captured outer iteration (no per-kernel events)")
    ap.add_argument("--schedule", type=str, default="0,1",
                    help="'auto' (autotuner), or CHUNK,STREAMS applied to every shape class")
    ap.add_argument("--order", type=int, default=0,
                    help="workgroup order flags of passes A / C (1: pass A, 2: pass C grouped by XCD); "
                         "ignored with --schedule auto, which tunes it")
    ap.add_argument("--cpu-procs", type=int, default=0, help="oracle processes (0: min(16, cores))")
    ap.add_argument("--cpu-outer", type=int, default=6, help="outer iterations of each oracle slice")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 1 GiB device copy before timing (HBM counter calibration under rocprof)")
    ap.add_argument("--gen-workers", type=int, default=0,
                    help="processes for input synthesis (0: auto); use 1 under a profiler (no fork)")
    ap.add_argument("--fast-data", action="store_true",
                    help="random inputs of the workload's shapes (same masks) instead of the phantom; "
                         "for counter runs only: the solver's memory traffic does not depend on values")
    ap.add_argument("--outer", type=int, default=0,
                    help="override the workload's outer iteration count (counter runs only; 0: the workload's)")
    ap.add_argument("--traffic", type=str,
                    default=os.path.join(ROOT, "profiles", "hbm_traffic_vol320_256x256_c8_t80_k4.json"),
                    help="rocprofv3 FETCH_SIZE / WRITE_SIZE summary (scaled HBM bytes per launch); ignored when "
                         "the kernel source or the workload differs from the one the counters were taken on")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU runs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    from synth import make_config

    t0 = time.perf_counter()
    if args.fast_data:
        d = make_config(args.config, max_slices=1, workers=1)
        rng = np.random.default_rng(0)
        for ci, c in enumerate(d["classes"]):
            n = d["cfg"]["classes"][ci]["nslices"]
            P = c.ksp.shape[2]
            c.sens = (rng.standard_normal((n, c.ncoils, c.ny, c.nz)).astype(np.float32) * (1 + 0j)).astype(np.complex64)
            c.sens /= np.sqrt((np.abs(c.sens) ** 2).sum(1, keepdims=True)).astype(np.float32)
            c.ksp = (rng.standard_normal((n, c.ncoils, P)) + 1j * rng.standard_normal((n, c.ncoils, P))).astype(np.complex64)
            c.slice_index = np.arange(n)
            log(f"class {ci}: random inputs for {n} slices")
    else:
        d = make_config(args.config, workers=args.gen_workers or None)
    cfg, phi = d["cfg"], d["phi"]
    classes = d["classes"]
    log(f"generated {cfg['name']} in {time.perf_counter() - t0:.1f} s")

    cpu = None
    if not args.no_cpu_baseline and not args.fast_data:
        nprocs = args.cpu_procs or min(16, os.cpu_count() or 1)
        cpu = cpu_baseline(classes[0], phi, cfg, nprocs, args.cpu_outer)
        log(f"cpu baseline: {cpu['value']:.4f} slices/s ({cpu['sample']})")

    if args.outer:
        cfg["n_outer"] = args.outer

    import torch

    import paper_1809_04195_amd as T
    from paper_1809_04195_amd.traffic_model import alg_bytes_per_slice

    assert torch.cuda.is_available(), "no GPU"
    dev = torch.device("cuda:0")
    plan = T.Plan(phi, [dict(ny=c.ny, nz=c.nz, ncoils=c.ncoils, nslices=c.nslices, masks=c.masks) for c in classes],
                  lam=cfg["lam"], rho=cfg["rho"], block=cfg["block"], n_outer=cfg["n_outer"], n_cg=cfg["n_cg"],
                  tol=cfg["tol"], seed=cfg["seed"])
    dsens = [torch.from_numpy(np.ascontiguousarray(c.sens)).to(dev) for c in classes]
    dksp = [torch.from_numpy(np.ascontiguousarray(c.ksp)).to(dev) for c in classes]
    torch.cuda.synchronize()
    log(f"workspace {plan.nbytes / 2**30:.2f} GiB, inputs resident in HBM")
    if args.copy_probe:
        a = torch.empty(2**28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy probe: 1 GiB read + 1 GiB write")
    mode = {"batched": T.T2S_BATCHED, "graph": T.T2S_BATCHED_GRAPH, "per_slice": T.T2S_PER_SLICE}[args.mode]
    stream = torch.cuda.current_stream()
    for ci in range(len(classes)):
        T.t2s_load_slices(plan.handle, ci, 0, classes[ci].nslices, dsens[ci], dksp[ci], stream)
    if args.schedule == "auto":
        t0 = time.perf_counter()
        T.t2s_autotune(plan.handle, 3, stream)
        log(f"autotune {time.perf_counter() - t0:.1f} s")
    else:
        ch, ns = (int(v) for v in args.schedule.split(","))
        for ci in range(len(classes)):
            T.t2s_set_schedule(plan.handle, ci, ch, ns)
            T.t2s_set_order(plan.handle, ci, args.order)
    scheds = [T.t2s_get_schedule(plan.handle, ci) for ci in range(len(classes))]
    orders = [T.t2s_get_order(plan.handle, ci) for ci in range(len(classes))]
    log(f"schedules (chunk, streams): {scheds}, workgroup orders {orders}")

    def step():
        for ci in range(len(classes)):
            T.t2s_load_slices(plan.handle, ci, 0, classes[ci].nslices, dsens[ci], dksp[ci], stream)
        T.t2s_reconstruct(plan.handle, mode, stream)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    T.t2s_profile_enable(plan.handle, mode != T.T2S_BATCHED_GRAPH)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        torch.cuda.synchronize()
        log(f"timed step {i + 1}/{args.steps} done at {time.perf_counter() - t0:.2f} s")
    elapsed = time.perf_counter() - t0
    prof = {name: T.t2s_profile_read(plan.handle, k) for k, name in enumerate(T.KERNEL_NAMES)}
    T.t2s_profile_enable(plan.handle, False)

    n_slices = sum(c.nslices for c in classes)
    ms_per_step = elapsed * 1000.0 / args.steps
    value = n_slices / (ms_per_step / 1000.0)

    # per kernel family: algorithmic bytes moved during the timed region / summed event time
    counts = {"pass_a": cfg["n_cg"], "pass_b": cfg["n_cg"], "pass_c": cfg["n_cg"], "llr_admm": 1}
    kern = {}
    for name, (n, ms) in prof.items():
        if n == 0:
            continue
        tb = None
        if name in counts:
            tb = sum(alg_bytes_per_slice(name, c.ny, c.nz, c.ncoils, phi.shape[1], cfg["n_cg"]) * c.nslices
                     for c in classes) * counts[name] * cfg["n_outer"] * args.steps
        kern[name] = dict(launches=n, total_ms=ms, avg_ms=ms / n,
                          alg_bytes_per_launch=(tb / n) if tb else None,
                          achieved_gbs=(tb / (ms * 1e6)) if tb else None)
    roofline = None
    if kern:
        dom = max((k for k in kern if kern[k]["alg_bytes_per_launch"]), key=lambda k: kern[k]["total_ms"])
        kd = kern[dom]
        traffic = None
        if args.traffic and os.path.exists(args.traffic):
            import hashlib
            tr = json.load(open(args.traffic))
            src = os.path.join(ROOT, "paper_1809_04195_amd", "csrc", "kernels.hip")
            cur = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
            same_sched = all(list(x) == [int(v) for v in tr.get("schedule", "0,1").split(",")] for x in scheds)
            same_sched = same_sched and all(o == tr.get("order", 0) for o in orders)
            if tr.get("kernels_source_sha256_16") == cur and tr.get("workload") == cfg["name"] and same_sched:
                t = tr["traffic"].get(dom)
                traffic = None if t is None else int(t["bytes_per_launch"])
        roofline = dict(bound="hbm", kernel=dom, achieved=round(kd["achieved_gbs"], 1), peak=HBM_PEAK_GBS,
                        unit="GB/s", frac=round(kd["achieved_gbs"] / HBM_PEAK_GBS, 4), traffic=traffic,
                        avg_launch_ms=round(kd["avg_ms"], 4), alg_bytes_per_launch=int(kd["alg_bytes_per_launch"]))
    # whole-solve algorithmic bandwidth (solver kernels with a byte model, per slice and outer iteration)
    per_outer = 0.0
    for c in classes:
        for name, mult in (("pass_a", cfg["n_cg"]), ("pass_b", cfg["n_cg"]), ("pass_c", cfg["n_cg"]),
                           ("llr_admm", 1)):
            per_outer += mult * c.nslices * alg_bytes_per_slice(name, c.ny, c.nz, c.ncoils, phi.shape[1], cfg["n_cg"])
    tot_bytes = per_outer * cfg["n_outer"] * args.steps
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "slices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "s_per_volume": round(ms_per_step / 1000.0, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "slices": n_slices,
                   "classes": [f"{c.nslices}x{c.ny}x{c.nz}c{c.ncoils}" for c in classes],
                   "T": int(phi.shape[0]), "K": int(phi.shape[1]), "outer": cfg["n_outer"], "cg": cfg["n_cg"],
                   "block": cfg["block"], "lambda": cfg["lam"], "rho": cfg["rho"], "mode": args.mode,
                   "step": "load_slices(device inputs) + reconstruct",
                   "schedules": [list(x) for x in scheds], "orders": orders},
        "roofline": roofline,
        "solver_alg_gbs": round(tot_bytes / (elapsed * 1e9), 1),
        "kernels": {k: dict(launches=v["launches"], avg_ms=round(v["avg_ms"], 4),
                            achieved_gbs=None if v["achieved_gbs"] is None else round(v["achieved_gbs"], 1))
                    for k, v in kern.items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
