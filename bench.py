"""Throughput of the T2-Shuffling slice reconstruction on one MI355X at equal ADMM
residual: plain solver vs batched launches + learned warm start.

Workload (default): the 512-slice 384 x 384 volume, C = 16 coils, T = 100 echoes,
K = 5, 1 % VD Poisson-disc sampling per echo, 8 x 8 LLR blocks, lambda = 0.01,
rho = 0.1, ADMM (5 CG per outer iteration) run to relative residual 1e-4 under the
shift-freeze stop rule, synthetic (seeded) data resident in HBM.

The volume is streamed through a plan of --slots slices (continuous batching,
t2s_stream_*): every slot holds one slice; at each stop decision the slots whose
slice stopped take the next slices of the volume (projection + adjoint of the
device-resident samples, the warm-start network on b0 = A^H y, the warm start), so
launches carry a full set of slices until the queue runs dry.  The timed region is
one whole volume, from empty slots to its last slice (every slice counted once, its
block shifts those of its global index): `steps` steps of ceil(512 / steps) completed
slices, the last one running until every slice has stopped.  The untimed warm-up
streams the first warmup x ceil(512 / steps) slices to completion.  `value` is
512 / the volume's time (slices/s); s/volume is that time.

Beside it, measured in the same run on two sampled batches of 32 slices: the plain
solver (one launch sequence per slice, cold start, same tolerance), the batched
solver (one 32-slice batch per launch) from a cold and from the network start, and
the streamed solver on the same slices; and the FP64 oracle on the host cores
(cpu_baseline), scaled by the plain run's outer-iteration count.  An extra 320-slice
256^2 volume run at the fixed 100 x 5 schedule gives the pass-B roofline at 256
points.  Prints one JSON line.

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


def solve_bytes(ny, nz, C, K, n_cg, slice_outer, n_warm):
    """Algorithmic bytes each kernel family moves for `slice_outer` outer iterations
    (summed over slices) plus `n_warm` warm starts (the normal operator of
    t2s_set_initial: pass A in its first-step form, pass B, pass C writing w)."""
    from paper_1809_04195_amd.traffic_model import alg_bytes_per_slice
    c8 = 8.0 * ny * nz
    its, n = float(slice_outer), float(n_warm)
    out = {k: its * n_cg * alg_bytes_per_slice(k, ny, nz, C, K, n_cg) for k in ("pass_a", "pass_b", "pass_c")}
    out["llr_admm"] = its * alg_bytes_per_slice("llr_admm", ny, nz, C, K, n_cg)
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
                     alg_bytes_per_launch=None if v["alg_bytes_per_launch"] is None else int(v["alg_bytes_per_launch"]),
                     achieved_gbs=None if v["achieved_gbs"] is None else round(v["achieved_gbs"], 1))
             for k, v in kern.items()}
    return roof, short


def counter_traffic(path, workload, kernel):
    """(HBM bytes per launch, their ratio to the algorithmic bytes of the same launches)
    of `kernel` from a committed counter summary, if it was taken on the current kernel
    source and this workload (else (None, None))."""
    import hashlib
    if not path or not os.path.exists(path):
        return None, None
    tr = json.load(open(path))
    src = os.path.join(ROOT, "paper_1809_04195_amd", "csrc", "kernels.hip")
    cur = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if tr.get("kernels_source_sha256_16") != cur or tr.get("workload") != workload:
        return None, None
    t = tr["traffic"].get(kernel)
    if t is None:
        return None, None
    r = t.get("ratio_to_alg")
    return int(t["bytes_per_launch"]), None if r is None else round(r, 3)


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
    T.t2s_profile_enable(plan.handle, False)
    alg = solve_bytes(cl.ny, cl.nz, cl.ncoils, phi.shape[1], cfg["n_cg"], cfg["n_outer"] * cl.nslices * steps, 0)
    roof, kern = roofline_from(prof, alg)
    roof["traffic"], roof["traffic_vs_alg"] = counter_traffic(
        os.path.join(ROOT, "profiles", "hbm_traffic_vol320_256x256_c8_t80_k4.json"), cfg["name"], roof["kernel"])
    plan.close()
    return dict(workload=cfg["name"], schedule="100 outer x 5 CG, batched", slices_per_s=round(
        cl.nslices * steps / el, 2), s_per_volume=round(el / steps, 4), roofline=roof, kernels=kern)


# ---------------------------------------------------------------------------


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=32, help="slices per batch of the comparison runs")
    ap.add_argument("--per-step", type=int, default=0,
                    help="slices completed per step (0: ceil(volume / steps), so that the timed steps cover one "
                         "volume and its mix of easy and hard slices)")
    ap.add_argument("--slots", type=int, default=256, help="slices the streaming plan holds at once")
    ap.add_argument("--queue-order", choices=("index", "energy"), default="index",
                    help="order the volume's slices are queued in: slice index, or descending sample energy (a "
                         "longest-first guess; it measured no faster on this volume)")
    ap.add_argument("--schedule", type=str, default="0,1",
                    help="CHUNK,STREAMS of the pass launches (0,1: all slots per launch on one stream, so every "
                         "kernel event times one whole launch), or 'auto' (the autotuner)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the classes' default kernel schedule flags (short counter runs under rocprofv3)")
    ap.add_argument("--plain-batches", type=str, default="4,11",
                    help="batches (of --batch slices) run with the plain, the batched and the streamed solver")
    ap.add_argument("--cpu-procs", type=int, default=0, help="oracle processes (0: min(16, cores))")
    ap.add_argument("--cpu-outer", type=int, default=2, help="outer iterations of each oracle slice")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-vol320", action="store_true", help="skip the 256^2 fixed-schedule extra")
    ap.add_argument("--vol320-steps", type=int, default=2)
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
    d = make_config("vol512_384x384_c16_t100_k5")
    cfg, phi = d["cfg"], d["phi"]
    cl = d["classes"][0]
    S, B, K, ncg, P = cl.nslices, args.batch, phi.shape[1], cfg["n_cg"], args.slots
    D = args.per_step or -(-S // args.steps)
    log(f"generated {cfg['name']} in {time.perf_counter() - t0:.1f} s")
    d320 = None
    if not args.no_vol320:
        t1 = time.perf_counter()
        d320 = make_config("vol320_256x256_c8_t80_k4")      # synthesised before the GPU is initialised (forked workers)
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
    log("copying the volume's coil maps and samples to the GPU")
    dsens = torch.from_numpy(cl.sens).to(dev)
    dksp = torch.from_numpy(cl.ksp).to(dev)
    torch.cuda.synchronize()
    net = T.UNet(K, 32, 4, max_batch=16, H=cl.ny, W=cl.nz)
    net.set_params(np.load(args.weights))

    def make_plan(n):
        return T.Plan(phi, [dict(ny=cl.ny, nz=cl.nz, ncoils=cl.ncoils, nslices=n, masks=cl.masks)], lam=cfg["lam"],
                      rho=cfg["rho"], block=cfg["block"], n_outer=cfg["n_outer"], n_cg=ncg, tol=cfg["tol"],
                      seed=cfg["seed"], **TOL_KW)

    def tune(plan, n):
        # schedule: autotuned (chunking over streams, kernel schedule flags) or fixed; the
        # flags are tuned unless --no-autotune (on the first n slices, loaded for it)
        if not args.no_autotune:
            T.t2s_load_slices(plan.handle, 0, 0, n, dsens[:n], dksp[:n], stream)
            T.t2s_autotune(plan.handle, 2, stream)
        if args.schedule != "auto":
            ch, ns = (int(v) for v in args.schedule.split(","))
            T.t2s_set_schedule(plan.handle, 0, ch, ns)
        return T.t2s_get_schedule(plan.handle, 0), T.t2s_get_order(plan.handle, 0)

    bplan, splan = make_plan(B), make_plan(P)
    log("plans bound; " + ("fixed schedule" if args.no_autotune else "autotuning"))
    t1 = time.perf_counter()
    tune(bplan, B)
    sched, order = tune(splan, P)
    log(f"volume inputs resident in HBM ({(dsens.numel() + dksp.numel()) * 8 / 2**30:.1f} GiB); workspaces "
        f"{bplan.nbytes / 2**30:.1f} GiB ({B}-slice batches), {splan.nbytes / 2**30:.1f} GiB ({P} streaming slots); "
        f"autotune {time.perf_counter() - t1:.1f} s: streaming schedule {sched}, order {order}")
    a0 = torch.empty((B, K, cl.ny, cl.nz), dtype=torch.complex64, device=dev)

    def run_batch(b, start, mode):
        first = b * B
        n = min(B, S - first)
        T.t2s_set_slice_offset(bplan.handle, 0, first)
        T.t2s_load_slices(bplan.handle, 0, 0, n, dsens[first:first + n], dksp[first:first + n], stream)
        if start == "net":
            b0 = bplan.read(0, 0, n, T.T2S_ADJOINT, device=True)
            for i in range(0, n, 16):
                net.forward(b0[i:i + 16], a0[i:i + 16])
            T.t2s_set_initial(bplan.handle, 0, 0, n, a0[:n], stream)
        T.t2s_reconstruct(bplan.handle, mode, stream)
        return n, [T.t2s_get_slice_report(bplan.handle, 0, s)["outer_iterations"] for s in range(n)]

    # the sampled batches: plain (per-slice launches, cold), batched cold, batched warm,
    # streamed warm (the batches' slices through the streaming plan)
    pb = [int(x) for x in args.plain_batches.split(",") if x]
    cmp = {}
    for key, start, mode in (("plain", "cold", T.T2S_PER_SLICE), ("batched_cold", "cold", T.T2S_BATCHED),
                             ("batched_warm", "net", T.T2S_BATCHED)):
        el, outer = 0.0, []
        for b in pb:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            n, its = run_batch(b, start, mode)
            torch.cuda.synchronize()
            el += time.perf_counter() - t1
            outer += its
            log(f"{key}: batch {b} ({n} slices) done, mean outer {np.mean(its):.1f}")
        cmp[key] = dict(s=el, slices=len(outer), outer=outer)
    if pb:
        # streamed through the batch plan's slots (a plan sized to the job: the
        # workgroup order deals contiguous slot ranges to the XCDs, so a few slices in
        # a large plan would use only some of them)
        out_cmp = torch.empty((len(pb) * B, K, cl.ny, cl.nz), dtype=torch.complex64, device=dev)
        bplan.stream_open(net, T.T2S_BATCHED)
        reps = [bplan.stream_submit(dsens[b * B:(b + 1) * B], dksp[b * B:(b + 1) * B], out_cmp[i * B:(i + 1) * B],
                                    b * B) for i, b in enumerate(pb)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        bplan.stream_run(0)
        torch.cuda.synchronize()
        outer = [r["outer_iterations"] for rep in reps for r in T.Plan.stream_reports(rep)]
        cmp["streamed_warm"] = dict(s=time.perf_counter() - t1, slices=len(outer), outer=outer)
        bplan.stream_close()
        log(f"streamed_warm: batches {pb} through {B} slots done, mean outer {np.mean(outer):.1f}")
        del out_cmp

    if args.copy_probe:
        ca = torch.empty(2**28, dtype=torch.float32, device=dev)
        cb = torch.empty_like(ca)
        cb.copy_(ca)
        torch.cuda.synchronize()
        del ca, cb
        log("copy probe: 1 GiB read + 1 GiB write")

    # warm-up (untimed): the first warmup x D slices of the volume streamed to completion
    out_vol = torch.empty((S, K, cl.ny, cl.nz), dtype=torch.complex64, device=dev)
    nw = min(S, args.warmup * D)
    if nw:
        splan.stream_open(net, T.T2S_BATCHED)
        splan.stream_submit(dsens[:nw], dksp[:nw], out_vol[:nw], 0)
        for i in range(args.warmup):
            _, st = splan.stream_run(D if i + 1 < args.warmup else 0)
            torch.cuda.synchronize()
            log(f"warmup step {i + 1}/{args.warmup}: {st['done']} of {nw} slices completed")
    # timed: the whole volume, from empty slots to its last slice, in `steps` steps of D
    # completed slices (the last step runs until every slice has stopped)
    splan.stream_open(net, T.T2S_BATCHED)
    if args.queue_order == "energy":
        # longest first: slices in descending order of their sample energy ||y||, a cost
        # proxy (slices without signal stop at the first check, the central ones take the
        # most outer iterations), so the volume does not end on its hardest slices
        energy = torch.linalg.vector_norm(dksp.reshape(S, -1), dim=1)
        queue = torch.argsort(energy, descending=True).cpu().numpy()
    else:
        queue = np.arange(S)
    rep = [splan.stream_submit(dsens[g:g + 1], dksp[g:g + 1], out_vol[g:g + 1], int(g)) for g in queue]
    T.t2s_profile_enable(splan.handle, True)
    torch.cuda.synchronize()
    st = dict(done=0, in_flight=S, loaded=0, slice_outer=0)
    t0 = time.perf_counter()
    for i in range(args.steps):
        code, st = splan.stream_run(max(1, (i + 1) * D - st["done"]) if i + 1 < args.steps else 0)
        torch.cuda.synchronize()
        log(f"timed step {i + 1}/{args.steps} done at {time.perf_counter() - t0:.2f} s: {st['done']} of {S} slices "
            f"completed")
        if st["in_flight"] == 0:
            break
    elapsed = time.perf_counter() - t0
    assert st["done"] == S and st["in_flight"] == 0, st
    prof = {name: T.t2s_profile_read(splan.handle, k) for k, name in enumerate(T.KERNEL_NAMES)}
    T.t2s_profile_enable(splan.handle, False)
    splan.stream_close()
    reps_vol = [T.Plan.stream_reports(r)[0] for r in rep]
    outer_vol = [r["outer_iterations"] for r in reps_vol]
    slices_done, slice_outer, loads = S, st["slice_outer"], st["loaded"]
    value = slices_done / elapsed
    alg = solve_bytes(cl.ny, cl.nz, cl.ncoils, K, ncg, slice_outer, loads)
    roof, kern = roofline_from(prof, alg)
    roof["traffic"], roof["traffic_vs_alg"] = counter_traffic(args.traffic, cfg["name"], roof["kernel"])
    solver_bytes = sum(alg.values())

    comp = None
    if pb:
        ns = cmp["plain"]["slices"]
        comp = dict(batches=pb, slices=ns, **{k: dict(slices_per_s=round(ns / v["s"], 3),
                                                      mean_outer=round(float(np.mean(v["outer"])), 1))
                                           for k, v in cmp.items()})
        comp["speedup_vs_plain"] = round(cmp["plain"]["s"] / cmp["streamed_warm"]["s"], 3)
        comp["speedup_batched_warm_vs_plain"] = round(cmp["plain"]["s"] / cmp["batched_warm"]["s"], 3)
        comp["speedup_warm_vs_cold"] = round(cmp["batched_cold"]["s"] / cmp["batched_warm"]["s"], 3)
    mean_cold_outer = float(np.mean(cmp["plain"]["outer"])) if pb else None
    bplan.close()
    splan.close()
    net.close()
    del dsens, dksp, out_vol
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
        "config": {"workload": cfg["name"], "slices": S, "slices_per_step": D, "T": int(phi.shape[0]), "K": int(K),
                   "coils": cl.ncoils, "grid": [cl.ny, cl.nz], "tol": cfg["tol"], "outer_cap": cfg["n_outer"],
                   "cg": ncg, "block": cfg["block"], "lambda": cfg["lam"], "rho": cfg["rho"],
                   "start": "warm (U-Net on b0)",
                   "mode": f"streamed through {P} slots (continuous batching, kernel events), queued by "
                           f"{'descending sample energy' if args.queue_order == 'energy' else 'slice index'}",
                   "step": f"{D} more slices of the volume completed (the last step: the rest): refills (load + "
                           "U-Net + warm start) and outer iterations to tolerance",
                   "comparison_batch": B,
                   "schedule": list(sched), "order": order},
        "roofline": roof,
        "solver_alg_gbs": round(solver_bytes / (elapsed * 1e9), 1),
        "slices_completed": slices_done,
        "mean_outer_warm": round(float(np.mean(outer_vol)), 1),
        "max_outer_warm": int(max(outer_vol)),
        "converged": int(sum(r["converged"] for r in reps_vol)),
        "kernels": kern,
        "comparison": comp,
        "vol320_fixed": extra,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
