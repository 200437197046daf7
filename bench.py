"""Throughput of the T2-Shuffling slice reconstruction on one MI355X at equal ADMM
residual: plain solver vs batched launches + learned warm start.

Workload (default): the 512-slice 384 x 384 volume, C = 16 coils, T = 100 echoes,
K = 5, 1 % VD Poisson-disc sampling per echo, 8 x 8 LLR blocks, lambda = 0.01,
rho = 0.1, ADMM (5 CG per outer iteration) run to relative residual 1e-4 under the
shift-freeze stop rule, synthetic (seeded) data resident in HBM.

One step = one batch of 32 consecutive readout slices of the volume (the next batch
each step, cycling through the volume; every slice keeps its global index, so its
block shifts are those of a whole-volume run): projection + adjoint of the
device-resident samples (t2s_load_slices), the warm-start network on b0 = A^H y
(t2s_unet_forward), the warm start (t2s_set_initial) and the ADMM solve to tolerance
(t2s_reconstruct, all 32 slices per launch, kernel events on).  `value` is slices/s
over the timed steps; s/volume = 512 / value.

Beside it, measured in the same run on two sampled batches: the plain solver (one
launch sequence per slice, cold start, same tolerance) and the batched solver from
a cold start, and the FP64 oracle on the host cores (cpu_baseline), scaled by the
plain run's outer-iteration count.  An extra 320-slice 256^2 volume run at the fixed
100 x 5 schedule gives the pass-B roofline at 256 points.  Prints one JSON line.

The network parameters come from paper_1809_04195_amd/weights/ (written by
python -m paper_1809_04195_amd.warmstart --workload vol512 --train-only).
"""

from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "readout slices/s & s/volume at equal ADMM residual: plain vs batched+warm-start"
HBM_PEAK_GBS = 8000.0
WEIGHTS = os.path.join(ROOT, "paper_1809_04195_amd", "weights", "unet_vol512_384x384_k5.npy")
TOL_KW = dict(freeze_window=5, freeze_stall=0.05, check_every=5)


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


def cpu_baseline(cl, phi, cfg, n_procs, outer, outer_to_tol=None):
    """Run the oracle on n_procs slices for `outer` outer iterations each, in parallel,
    and scale to complete solves: cfg's n_outer iterations, or `outer_to_tol` (the mean
    outer iterations a cold start needs to reach the tolerance) when given."""
    sel = np.linspace(0, cl.nslices - 1, n_procs).round().astype(int)
    _CPU.update(ksp=cl.ksp[sel], sens=cl.sens[sel], phi=phi, masks=cl.masks.astype(bool), lam=cfg["lam"],
                rho=cfg["rho"], block=cfg["block"], outer=outer, n_cg=cfg["n_cg"], seed=cfg["seed"], g=sel)
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(n_procs) as pool:
        per = pool.map(_oracle_job, range(n_procs))
    wall = time.perf_counter() - t0
    need = outer_to_tol if outer_to_tol else cfg["n_outer"]
    frac = outer / need
    what = (f"{need:.1f} outer iterations (the mean a cold start needs to reach the tolerance)" if outer_to_tol
            else f"{cfg['n_outer']} ADMM outer iterations")
    return dict(value=n_procs * frac / wall, unit="slices/s", cores=n_procs, kind="oracle",
                sample=f"{n_procs} slices x {outer} of {what} (5 CG), FP64 NumPy, one process per slice, "
                       f"wall {wall:.1f} s, per-slice {np.mean(per):.1f} s",
                s_per_volume=cl.nslices / (n_procs * frac / wall))


# ---------------------------------------------------------------------------
# algorithmic bytes of a tolerance run (per kernel family)
# ---------------------------------------------------------------------------


def tolerance_run_bytes(ny, nz, C, K, n_cg, outer_iters, warm):
    """Algorithmic bytes each kernel family moves for slices that ran `outer_iters`
    outer iterations (plus, for a warm start, the normal operator of t2s_set_initial)."""
    from paper_1809_04195_amd.traffic_model import alg_bytes_per_slice
    c8 = 8.0 * ny * nz
    its = float(np.sum(outer_iters))
    n = len(outer_iters)
    out = {k: its * n_cg * alg_bytes_per_slice(k, ny, nz, C, K, n_cg) for k in ("pass_a", "pass_b", "pass_c")}
    out["llr_admm"] = its * alg_bytes_per_slice("llr_admm", ny, nz, C, K, n_cg)
    if warm:   # normal operator on alpha0: pass A (first-step form), pass B, pass C writing w
        out["pass_a"] += n * c8 * (2 * K + C + C * K)
        out["pass_b"] += n * alg_bytes_per_slice("pass_b", ny, nz, C, K, n_cg)
        out["pass_c"] += n * c8 * (C * K + C + 2 * K)
    return out


def roofline_from(prof, alg):
    """Per kernel family: launches, average time, algorithmic GB/s; and the roofline
    object of the family with the largest total time."""
    kern = {}
    for name, (n, ms) in prof.items():
        if n == 0:
            continue
        b = alg.get(name)
        kern[name] = dict(launches=n, total_ms=ms, avg_ms=ms / n, alg_bytes_per_launch=(b / n) if b else None,
                          achieved_gbs=(b / (ms * 1e6)) if b else None)
    dom = max((k for k in kern if kern[k]["alg_bytes_per_launch"]), key=lambda k: kern[k]["total_ms"])
    kd = kern[dom]
    roof = dict(bound="hbm", kernel=dom, achieved=round(kd["achieved_gbs"], 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(kd["achieved_gbs"] / HBM_PEAK_GBS, 4), traffic=None,
                avg_launch_ms=round(kd["avg_ms"], 4), alg_bytes_per_launch=int(kd["alg_bytes_per_launch"]))
    short = {k: dict(launches=v["launches"], avg_ms=round(v["avg_ms"], 4),
                     achieved_gbs=None if v["achieved_gbs"] is None else round(v["achieved_gbs"], 1))
             for k, v in kern.items()}
    return roof, short


def counter_traffic(path, workload, kernel):
    """HBM bytes per launch of `kernel` from a committed counter summary, if it was taken
    on the current kernel source and this workload (else None)."""
    import hashlib
    if not path or not os.path.exists(path):
        return None
    tr = json.load(open(path))
    src = os.path.join(ROOT, "paper_1809_04195_amd", "csrc", "kernels.hip")
    cur = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if tr.get("kernels_source_sha256_16") != cur or tr.get("workload") != workload:
        return None
    t = tr["traffic"].get(kernel)
    return None if t is None else int(t["bytes_per_launch"])


# ---------------------------------------------------------------------------
# the 256^2 fixed-schedule volume (pass-B roofline at 256 points)
# ---------------------------------------------------------------------------


def fixed_vol320(T, torch, d, steps):
    cfg, phi, cl = d["cfg"], d["phi"], d["classes"][0]
    plan = T.Plan(phi, [dict(ny=cl.ny, nz=cl.nz, ncoils=cl.ncoils, nslices=cl.nslices, masks=cl.masks)],
                  lam=cfg["lam"], rho=cfg["rho"], block=cfg["block"], n_outer=cfg["n_outer"], n_cg=cfg["n_cg"],
                  seed=cfg["seed"])
    ds = torch.from_numpy(cl.sens).cuda()
    dk = torch.from_numpy(cl.ksp).cuda()
    stream = torch.cuda.current_stream()

    def step():
        T.t2s_load_slices(plan.handle, 0, 0, cl.nslices, ds, dk, stream)
        T.t2s_reconstruct(plan.handle, T.T2S_BATCHED, stream)

    step()
    torch.cuda.synchronize()
    T.t2s_profile_enable(plan.handle, True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = {name: T.t2s_profile_read(plan.handle, k) for k, name in enumerate(T.KERNEL_NAMES)}
    alg = tolerance_run_bytes(cl.ny, cl.nz, cl.ncoils, phi.shape[1], cfg["n_cg"],
                              [cfg["n_outer"]] * cl.nslices * steps, False)
    roof, kern = roofline_from(prof, alg)
    roof["traffic"] = counter_traffic(os.path.join(ROOT, "profiles", "hbm_traffic_vol320_256x256_c8_t80_k4.json"),
                                      cfg["name"], roof["kernel"])
    plan.close()
    return dict(workload=cfg["name"], schedule="100 outer x 5 CG, batched", slices_per_s=round(
        cl.nslices * steps / el, 2), s_per_volume=round(el / steps, 4), roofline=roof, kernels=kern)


# ---------------------------------------------------------------------------


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=32, help="slices per step")
    ap.add_argument("--schedule", type=str, default="0,1",
                    help="CHUNK,STREAMS of the pass launches (0,1: all slices of a step per launch on one stream, "
                         "so every kernel event times one whole launch), or 'auto' (the autotuner; its multi-stream "
                         "schedules overlap launches, which stretches the per-launch event times)")
    ap.add_argument("--plain-batches", type=str, default="4,11",
                    help="batches (of --batch slices) run with the plain and the cold batched solver")
    ap.add_argument("--cpu-procs", type=int, default=0, help="oracle processes (0: min(16, cores))")
    ap.add_argument("--cpu-outer", type=int, default=2, help="outer iterations of each oracle slice")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-vol320", action="store_true", help="skip the 256^2 fixed-schedule extra")
    ap.add_argument("--vol320-steps", type=int, default=2)
    ap.add_argument("--first-batch", type=int, default=0,
                    help="batch of the first warm-up step (the steps then go through the volume in order)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 1 GiB device copy before timing (HBM counter calibration under rocprof)")
    ap.add_argument("--weights", type=str, default=WEIGHTS)
    ap.add_argument("--traffic", type=str,
                    default=os.path.join(ROOT, "profiles", "hbm_traffic_vol512_384x384_c16_t100_k5.json"),
                    help="rocprofv3 FETCH_SIZE / WRITE_SIZE summary (scaled HBM bytes per launch); ignored when "
                         "the kernel source or the workload differs from the one the counters were taken on")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU runs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if not os.path.exists(args.weights):
        raise SystemExit(f"warm-start network parameters {args.weights} are missing: train them with "
                         "python -m paper_1809_04195_amd.warmstart --workload vol512 --train-only")

    from synth import make_config

    t0 = time.perf_counter()
    d = make_config(4)
    cfg, phi = d["cfg"], d["phi"]
    cl = d["classes"][0]
    S, B, K, ncg = cl.nslices, args.batch, phi.shape[1], cfg["n_cg"]
    nb = (S + B - 1) // B
    log(f"generated {cfg['name']} in {time.perf_counter() - t0:.1f} s")
    d320 = None
    if not args.no_vol320:
        t1 = time.perf_counter()
        d320 = make_config(1)      # synthesised before the GPU is initialised (forked workers)
        log(f"generated {d320['cfg']['name']} in {time.perf_counter() - t1:.1f} s")

    # the oracle runs before the GPU is initialised (its workers are forked); its time
    # per outer iteration is scaled to a whole solve once the plain run has measured
    # the outer iterations a cold start needs
    cpu_raw = None
    if not args.no_cpu_baseline:
        nprocs = args.cpu_procs or min(16, os.cpu_count() or 1)
        cpu_raw = cpu_baseline(cl, phi, cfg, nprocs, args.cpu_outer)
        log(f"cpu baseline sample: {cpu_raw['sample']}")

    import torch

    import paper_1809_04195_amd as T

    assert torch.cuda.is_available(), "no GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    dsens = torch.from_numpy(cl.sens).to(dev)
    dksp = torch.from_numpy(cl.ksp).to(dev)
    torch.cuda.synchronize()
    net = T.UNet(K, 32, 4, max_batch=16, H=cl.ny, W=cl.nz)
    net.set_params(np.load(args.weights))
    plan = T.Plan(phi, [dict(ny=cl.ny, nz=cl.nz, ncoils=cl.ncoils, nslices=B, masks=cl.masks)], lam=cfg["lam"],
                  rho=cfg["rho"], block=cfg["block"], n_outer=cfg["n_outer"], n_cg=ncg, tol=cfg["tol"],
                  seed=cfg["seed"], **TOL_KW)
    a0 = torch.empty((B, K, cl.ny, cl.nz), dtype=torch.complex64, device=dev)
    log(f"volume inputs resident in HBM ({(dsens.numel() + dksp.numel()) * 8 / 2**30:.1f} GiB), "
        f"plan workspace {plan.nbytes / 2**30:.1f} GiB for {B} slices")

    def run_batch(b, start, mode):
        first = b * B
        n = min(B, S - first)
        T.t2s_set_slice_offset(plan.handle, 0, first)
        T.t2s_load_slices(plan.handle, 0, 0, n, dsens[first:first + n], dksp[first:first + n], stream)
        if start == "net":
            b0 = plan.read(0, 0, n, T.T2S_ADJOINT, device=True)
            for i in range(0, n, 16):
                net.forward(b0[i:i + 16], a0[i:i + 16])
            T.t2s_set_initial(plan.handle, 0, 0, n, a0[:n], stream)
        code = T.t2s_reconstruct(plan.handle, mode, stream)
        return code, n

    def reports(n):
        return [T.t2s_get_slice_report(plan.handle, 0, s) for s in range(n)]

    # schedule: autotuned (chunking over streams, workgroup order) or fixed; the
    # workgroup order is always tuned
    T.t2s_load_slices(plan.handle, 0, 0, B, dsens[:B], dksp[:B], stream)
    t1 = time.perf_counter()
    T.t2s_autotune(plan.handle, 2, stream)
    if args.schedule != "auto":
        ch, ns = (int(v) for v in args.schedule.split(","))
        T.t2s_set_schedule(plan.handle, 0, ch, ns)
    sched, order = T.t2s_get_schedule(plan.handle, 0), T.t2s_get_order(plan.handle, 0)
    log(f"autotune {time.perf_counter() - t1:.1f} s: schedule {sched}, order {order}")

    # plain (per-slice launches, cold) and batched cold on the sampled batches
    pb = [int(x) for x in args.plain_batches.split(",") if x]
    cmp = {"plain": {}, "cold": {}}
    for key, mode in (("plain", T.T2S_PER_SLICE), ("cold", T.T2S_BATCHED)):
        for b in pb:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            code, n = run_batch(b, "cold", mode)
            torch.cuda.synchronize()
            el = time.perf_counter() - t1
            its = [r["outer_iterations"] for r in reports(n)]
            cmp[key][b] = dict(s=el, slices=n, outer=its, code=code)
            log(f"{key}: batch {b} ({n} slices) in {el:.2f} s, mean outer {np.mean(its):.1f}")

    if args.copy_probe:
        ca = torch.empty(2**28, dtype=torch.float32, device=dev)
        cb = torch.empty_like(ca)
        cb.copy_(ca)
        torch.cuda.synchronize()
        del ca, cb
        log("copy probe: 1 GiB read + 1 GiB write")
    for i in range(args.warmup):
        run_batch((args.first_batch + i) % nb, "net", T.T2S_BATCHED)
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    T.t2s_profile_enable(plan.handle, True)
    torch.cuda.synchronize()
    steps = []
    t0 = time.perf_counter()
    tprev = t0
    for i in range(args.steps):
        b = (args.first_batch + args.warmup + i) % nb
        code, n = run_batch(b, "net", T.T2S_BATCHED)
        torch.cuda.synchronize()
        now = time.perf_counter()
        steps.append(dict(batch=b, s=now - tprev, slices=n, code=code, outer=[r["outer_iterations"] for r in reports(n)]))
        tprev = time.perf_counter()
        log(f"timed step {i + 1}/{args.steps} (batch {b}) done at {now - t0:.2f} s, "
            f"mean outer {np.mean(steps[-1]['outer']):.1f}")
    elapsed = time.perf_counter() - t0
    prof = {name: T.t2s_profile_read(plan.handle, k) for k, name in enumerate(T.KERNEL_NAMES)}
    T.t2s_profile_enable(plan.handle, False)
    slices_done = sum(s["slices"] for s in steps)
    value = slices_done / elapsed
    its_all = [x for s in steps for x in s["outer"]]
    alg = tolerance_run_bytes(cl.ny, cl.nz, cl.ncoils, K, ncg, its_all, True)
    roof, kern = roofline_from(prof, alg)
    roof["traffic"] = counter_traffic(args.traffic, cfg["name"], roof["kernel"])
    solver_bytes = sum(alg.values())

    # plain vs batched + warm start on the same batches (timed steps that covered them)
    warm_on = {}
    for s in steps:
        if s["batch"] in pb and s["batch"] not in warm_on:
            warm_on[s["batch"]] = s
    comp = None
    if pb and all(b in warm_on for b in pb):
        tp = sum(cmp["plain"][b]["s"] for b in pb)
        tc = sum(cmp["cold"][b]["s"] for b in pb)
        tw = sum(warm_on[b]["s"] for b in pb)
        ns = sum(cmp["plain"][b]["slices"] for b in pb)
        comp = dict(batches=pb, slices=ns,
                    plain=dict(slices_per_s=round(ns / tp, 3), mean_outer=round(float(np.mean(
                        [x for b in pb for x in cmp["plain"][b]["outer"]])), 1)),
                    batched_cold=dict(slices_per_s=round(ns / tc, 3), mean_outer=round(float(np.mean(
                        [x for b in pb for x in cmp["cold"][b]["outer"]])), 1)),
                    batched_warm=dict(slices_per_s=round(ns / tw, 3), mean_outer=round(float(np.mean(
                        [x for b in pb for x in warm_on[b]["outer"]])), 1)),
                    speedup_vs_plain=round(tp / tw, 3), speedup_warm_vs_cold=round(tc / tw, 3))
    mean_cold_outer = float(np.mean([x for b in pb for x in cmp["plain"][b]["outer"]])) if pb else None
    plan.close()
    net.close()
    del dsens, dksp
    torch.cuda.empty_cache()

    extra = None
    if not args.no_vol320:
        t1 = time.perf_counter()
        extra = fixed_vol320(T, torch, d320, args.vol320_steps)
        log(f"256^2 fixed-schedule extra in {time.perf_counter() - t1:.1f} s")

    cpu = None
    if cpu_raw is not None:
        need = mean_cold_outer or cfg["n_outer"]
        scale = cfg["n_outer"] / need      # cpu_raw is scaled to n_outer iterations per slice
        cpu = dict(cpu_raw, value=cpu_raw["value"] * scale, s_per_volume=cpu_raw["s_per_volume"] / scale,
                   sample=cpu_raw["sample"].replace(f"{cfg['n_outer']} ADMM outer iterations",
                                                    f"{need:.1f} outer iterations (the mean the plain cold run "
                                                    f"needed to reach the tolerance)"))
        log(f"cpu baseline: {cpu['value']:.5f} slices/s ({cpu['sample']})")

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "slices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1000.0 / args.steps, 2),
        "s_per_volume": round(S / value, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "slices": S, "slices_per_step": B, "T": int(phi.shape[0]), "K": int(K),
                   "coils": cl.ncoils, "grid": [cl.ny, cl.nz], "tol": cfg["tol"], "outer_cap": cfg["n_outer"],
                   "cg": ncg, "block": cfg["block"], "lambda": cfg["lam"], "rho": cfg["rho"],
                   "start": "warm (U-Net on b0)", "mode": "batched (all slices of a step per launch, kernel events)",
                   "step": "load_slices(device inputs) + U-Net + set_initial + reconstruct to tol",
                   "schedule": list(sched), "order": order},
        "roofline": roof,
        "solver_alg_gbs": round(solver_bytes / (elapsed * 1e9), 1),
        "mean_outer_warm": round(float(np.mean(its_all)), 1),
        "kernels": kern,
        "comparison": comp,
        "vol320_fixed": extra,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
