"""Learned warm start for the slice solver: training pairs from the solver itself,
U-Net training on the GPU, and the equal-residual comparison of ADMM started cold,
from b0 = A^H y, and from the network's prediction.

Every numerical step runs in libt2s.so (solver and network kernels); this module
only moves data between the C entry points (PyTorch owns device memory).

    python -m paper_1809_04195_amd.warmstart --workload eval320
    python -m paper_1809_04195_amd.warmstart --workload vol512 --train-only
    python -m paper_1809_04195_amd.warmstart --workload vol512 --params <saved .npy> --plain
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import (T2S_ADJOINT, T2S_ALPHA, T2S_BATCHED, T2S_BATCHED_GRAPH, T2S_PER_SLICE, Plan, UNet, t2s_autotune,
               t2s_get_order, t2s_get_schedule, t2s_set_slice_offset)
from .traffic_model import bytes_per_outer


def log(msg):
    print(f"[warmstart] {msg}", flush=True)


# ---------------------------------------------------------------------------
# training pairs: (b0, alpha after the fixed 100 x 5 schedule) per slice
# ---------------------------------------------------------------------------


def solve_chunk(phi, masks, sens, ksp, ptot, mid, cfg, seed):
    """Reconstruct one chunk of training slices (one shape class per mask set).
    Returns device tensors (b0, alpha) [n, K, ny, nz] in chunk order."""
    import torch
    n = sens.shape[0]
    sets = sorted(set(int(m) for m in mid))
    groups = [np.flatnonzero(mid == m) for m in sets]
    ny, nz = masks.shape[2], masks.shape[3]
    classes = [dict(ny=ny, nz=nz, ncoils=sens.shape[1], nslices=len(g), masks=masks[m]) for m, g in zip(sets, groups)]
    plan = Plan(phi, classes, lam=cfg["lam"], rho=cfg["rho"], block=cfg["block"], n_outer=cfg["n_outer"],
                n_cg=cfg["n_cg"], seed=seed)
    for ci, g in enumerate(groups):
        P = int(ptot[g[0]])
        plan.load(ci, 0, np.ascontiguousarray(sens[g]), np.ascontiguousarray(ksp[g][:, :, :P]))
    plan.reconstruct(T2S_BATCHED_GRAPH)
    K = phi.shape[1]
    b0 = torch.empty((n, K, ny, nz), dtype=torch.complex64, device="cuda")
    alpha = torch.empty_like(b0)
    for ci, g in enumerate(groups):
        gi = torch.from_numpy(g).cuda()
        b0[gi] = plan.read(ci, 0, len(g), T2S_ADJOINT, device=True)
        alpha[gi] = plan.read(ci, 0, len(g), T2S_ALPHA, device=True)
    torch.cuda.synchronize()
    plan.close()
    return b0, alpha


def training_pairs(n, seed, mask_sets, phi, cfg, ny=256, nz=256, C=8, chunk=800):
    import torch
    from synth import make_training_chunk, training_masks

    t0 = time.perf_counter()
    masks = training_masks(seed, mask_sets, ny, nz, phi.shape[0], cfg["frac"])
    log(f"{mask_sets} mask sets of {ny}x{nz} in {time.perf_counter() - t0:.1f} s")
    b0s, als = [], []
    for first in range(0, n, chunk):
        m = min(chunk, n - first)
        t1 = time.perf_counter()
        sens, ksp, ptot, mid = make_training_chunk(first, m, seed, masks, C=C)
        t2 = time.perf_counter()
        b0, al = solve_chunk(phi, masks, sens, ksp, ptot, mid, cfg, seed + first)
        b0s.append(b0)
        als.append(al)
        log(f"training slices {first}..{first + m - 1}: synthesised {t2 - t1:.1f} s, solved {time.perf_counter() - t2:.1f} s")
        del sens, ksp
    return torch.cat(b0s), torch.cat(als)


# ---------------------------------------------------------------------------
# training
# ---------------------------------------------------------------------------


def train(net, b0, alpha, epochs, batch, lr, seed):
    import torch
    n = b0.shape[0]
    rng = np.random.default_rng(seed)
    hist = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = rng.permutation(n)
        lr_ep = lr * (0.5 * (1 + np.cos(np.pi * ep / epochs)))      # cosine decay
        losses = []
        for i in range(0, n - batch + 1, batch):
            idx = torch.from_numpy(perm[i:i + batch]).cuda()
            xb = b0[idx].contiguous()
            tb = alpha[idx].contiguous()
            want = (i // batch) % 25 == 0
            l = net.train_step(xb, tb, lr_ep, want_loss=want)
            if want:
                losses.append(l)
        torch.cuda.synchronize()
        hist.append(float(np.mean(losses)))
        log(f"epoch {ep + 1}/{epochs}: mean sampled loss {hist[-1]:.5f} (lr {lr_ep:.2e}) at {time.perf_counter() - t0:.1f} s")
    return hist, time.perf_counter() - t0


# ---------------------------------------------------------------------------
# equal-residual comparison
# ---------------------------------------------------------------------------


def _solve_group(phi, cl, cfg, start, net, batch, mode, first, count, tune):
    """Reconstruct slices [first, first + count) of the volume to tol in one plan whose
    slice 0 has global index `first` (same shifts as in a whole-volume plan).
    Returns (wall seconds of load + start + solve, reports, alpha, alpha0, schedule, order)."""
    import torch
    sl = slice(first, first + count)
    plan = Plan(phi, [dict(ny=cl.ny, nz=cl.nz, ncoils=cl.ncoils, nslices=count, masks=cl.masks)], lam=cfg["lam"],
                rho=cfg["rho"], block=cfg["block"], n_outer=cfg["n_outer"], n_cg=cfg["n_cg"], tol=cfg["tol"],
                seed=cfg["seed"], freeze_window=5, freeze_stall=0.05, check_every=5)
    t2s_set_slice_offset(plan.handle, 0, first)
    dsens = torch.from_numpy(np.ascontiguousarray(cl.sens[sl])).cuda()
    dksp = torch.from_numpy(np.ascontiguousarray(cl.ksp[sl])).cuda()
    if tune:
        plan.load(0, 0, dsens, dksp)
        t2s_autotune(plan.handle, 2)
    sched, order = t2s_get_schedule(plan.handle, 0), t2s_get_order(plan.handle, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.load(0, 0, dsens, dksp)
    a0 = None
    if start != "cold":
        b0 = plan.read(0, 0, count, T2S_ADJOINT, device=True)
        if start == "b0":
            a0 = b0
        else:
            a0 = torch.empty_like(b0)
            for i in range(0, count, batch):
                net.forward(b0[i:i + batch], a0[i:i + batch])
        plan.set_initial(0, 0, a0)
    code = plan.reconstruct(mode)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    reps = [plan.report(0, s) for s in range(count)]
    alpha = plan.read(0, 0, count, T2S_ALPHA, device=True)
    plan.close()
    return wall, reps, alpha, a0, sched, order, code


def run_tolerance(phi, cl, cfg, start, net=None, batch=16, mode=T2S_BATCHED_GRAPH, group=0):
    """Load, optionally warm start, reconstruct to tol.  start: 'cold' | 'b0' | 'net';
    mode: T2S_BATCHED_GRAPH (batched, autotuned) or T2S_PER_SLICE (one launch sequence
    per slice).  `group` > 0 runs the volume as consecutive plans of that many slices
    (each slice keeps its global index, so the arithmetic is unchanged) and reports the
    summed time; it is meant for the per-slice schedule, which gains nothing from
    having the whole volume in one plan."""
    import torch
    S = cl.nslices
    group = group or S
    wall, reps, alphas, a0s, code = 0.0, [], [], [], 0
    for first in range(0, S, group):
        n = min(group, S - first)
        w, r, a, a0, sched, order, c = _solve_group(phi, cl, cfg, start, net, batch, mode, first, n,
                                                    tune=mode != T2S_PER_SLICE)
        wall += w
        reps += r
        alphas.append(a)
        a0s.append(a0)
        code = max(code, int(c))
        if group < S:
            log(f"  {start} ({'per-slice' if mode == T2S_PER_SLICE else 'batched'}): slices {first}..{first + n - 1} "
                f"in {w:.1f} s")
    alpha = torch.cat(alphas)
    a0 = None if a0s[0] is None else torch.cat(a0s)
    its = np.array([r["outer_iterations"] for r in reps])
    alg = float(its.sum()) * bytes_per_outer(cl.ny, cl.nz, cl.ncoils, phi.shape[1], cfg["n_cg"])
    res = dict(start=start, mode="per_slice" if mode == T2S_PER_SLICE else "batched_graph", s_per_volume=wall,
               slices_per_s=S / wall, outer_mean=float(its.mean()), outer_max=int(its.max()), outer_min=int(its.min()),
               converged=int(sum(r["converged"] for r in reps)), slices=S, code=int(code),
               final_residual_max=float(max(max(r["r_primal"], r["r_dual"]) for r in reps)),
               solver_alg_gbs=alg / wall / 1e9, schedule=list(sched), order=order,
               plans=(S + group - 1) // group)
    return res, alpha, a0


# Workloads: the training geometry (2D phantoms, its own masks) follows the volume
# the network is evaluated on; targets are the fixed 100 x 5 schedule's solution.
WORKLOADS = {
    "eval320": dict(eval_workload="warmstart_eval320_256x256_c8_t80_k4", ny=256, nz=256, C=8, K=4, frac=0.015, chunk=800),
    "vol512": dict(eval_workload="vol512_384x384_c16_t100_k5", ny=384, nz=384, C=16, K=5, frac=0.01, chunk=200),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="eval320",
                    help="eval320: held-out 320-slice 256^2 C8 K4 volume; vol512: 512-slice 384^2 C16 T100 K5 volume")
    ap.add_argument("--train-slices", type=int, default=4000)
    ap.add_argument("--mask-sets", type=int, default=40)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--train-seed", type=int, default=10)
    ap.add_argument("--eval-slices", type=int, default=0, help="0: the whole volume")
    ap.add_argument("--out", type=str, default="")
    ap.add_argument("--save-params", type=str, default="")
    ap.add_argument("--save-samples", type=int, default=2, help="eval slices whose outputs are saved for oracle checks")
    ap.add_argument("--params", type=str, default="", help="trained parameters (.npy): skip data generation and training")
    ap.add_argument("--train-only", action="store_true", help="stop after training (parameters saved)")
    ap.add_argument("--plain", action="store_true", help="also run the plain solver: per-slice launches, cold start")
    ap.add_argument("--plain-group", type=int, default=32,
                    help="slices per plan of the plain run (progress is printed per plan)")
    ap.add_argument("--starts", type=str, default="cold,b0,net",
                    help="batched runs to make (comma list of cold, b0, net; empty with --plain: plain only)")
    args = ap.parse_args()
    wl = WORKLOADS[args.workload]
    args.out = args.out or f"warmstart_out/warmstart_{args.workload}.json"
    if not args.save_params:   # the parameters bench.py and the warm-start runs load
        args.save_params = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                                        f"unet_{args.workload}_{wl['ny']}x{wl['nz']}_k{wl['K']}.npy")
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)

    import torch

    from synth import CONFIGS, basis, make_config

    assert torch.cuda.is_available()
    ecfg = dict(CONFIGS[wl["eval_workload"]])
    tcfg = dict(ecfg, n_outer=100, n_cg=5, tol=0.0, frac=wl["frac"])      # schedule of the training targets
    phi = basis(ecfg["T"], ecfg["K"])
    K = phi.shape[1]
    ny, nz = wl["ny"], wl["nz"]
    out = dict(workload=args.workload,
               config=dict(train_slices=args.train_slices, mask_sets=args.mask_sets, epochs=args.epochs,
                           batch=args.batch, lr=args.lr, eval_slices=args.eval_slices or None, tol=ecfg["tol"],
                           grid=[ny, nz], coils=wl["C"], T=ecfg["T"], K=K))
    net = UNet(K, 32, 4, max_batch=args.batch, H=ny, W=nz)
    if args.params:
        net.set_params(np.load(args.params))
        out["train"] = dict(params=args.params)
    else:
        t0 = time.perf_counter()
        b0, alpha = training_pairs(args.train_slices, args.train_seed, args.mask_sets, phi, tcfg, ny=ny, nz=nz,
                                   C=wl["C"], chunk=wl["chunk"])
        out["pairs_s"] = time.perf_counter() - t0
        log(f"{args.train_slices} training pairs in {out['pairs_s']:.1f} s")
        net.set_params(net.init_params(args.train_seed))
        hist, ttrain = train(net, b0, alpha, args.epochs, args.batch, args.lr, args.train_seed)
        out["train"] = dict(loss_per_epoch=hist, seconds=ttrain,
                            slices_per_s=args.train_slices * args.epochs / ttrain)
        params = net.get_params()
        if args.save_params:
            os.makedirs(os.path.dirname(args.save_params) or ".", exist_ok=True)
            np.save(args.save_params, params)
        del b0, alpha
        torch.cuda.empty_cache()
        if args.train_only:
            json.dump(out, open(args.out, "w"), indent=1)
            log(json.dumps(out))
            net.close()
            return

    # held-out evaluation volume
    t0 = time.perf_counter()
    d = make_config(wl["eval_workload"], max_slices=args.eval_slices or None)
    cl = d["classes"][0]
    log(f"evaluation volume ({cl.nslices} x {cl.ny}x{cl.nz} C{cl.ncoils}) generated in {time.perf_counter() - t0:.1f} s")
    runs = {}
    sols = {}
    starts = [x for x in args.starts.split(",") if x]
    for start in starts:
        r, a, a0 = run_tolerance(phi, cl, ecfg, start, net)
        runs[start] = r
        sols[start] = (a, a0)
        log(f"{start}: {r}")

    def rel(x, y):
        return float(torch.linalg.vector_norm(x - y) / torch.linalg.vector_norm(y))

    out["eval"] = runs
    full = all(x in sols for x in ("cold", "b0", "net"))
    if full:
        ref = sols["cold"][0]
        a0n = sols["net"][1]
        out["start_error_vs_solution"] = dict(net=rel(a0n, ref), b0=rel(sols["b0"][1], ref), zero=1.0)
    if args.plain:
        r, _, _ = run_tolerance(phi, cl, ecfg, "cold", None, mode=T2S_PER_SLICE, group=args.plain_group)
        runs["plain"] = r
        log(f"plain (per-slice launches, cold): {r}")
        if full:
            out["speedup_batched_net_vs_plain"] = r["s_per_volume"] / runs["net"]["s_per_volume"]
            out["speedup_batched_cold_vs_plain"] = r["s_per_volume"] / runs["cold"]["s_per_volume"]
    if full:
        out["speedup_net_vs_cold"] = runs["cold"]["s_per_volume"] / runs["net"]["s_per_volume"]
        out["speedup_b0_vs_cold"] = runs["cold"]["s_per_volume"] / runs["b0"]["s_per_volume"]
        out["outer_saved_net_vs_cold"] = runs["cold"]["outer_mean"] - runs["net"]["outer_mean"]
    if args.save_samples and full:
        sel = np.linspace(0, cl.nslices - 1, args.save_samples + 2).round().astype(int)[1:-1]
        np.savez(os.path.splitext(args.out)[0] + "_samples.npz", slices=sel,
                 index=cl.slice_index[sel], net=a0n[sel].cpu().numpy(), solution=ref[sel].cpu().numpy())
    json.dump(out, open(args.out, "w"), indent=1)
    log(json.dumps(out))
    net.close()


if __name__ == "__main__":
    main()
