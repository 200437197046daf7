"""Batching of slices of uneven size: the mixed 48-slice batch (16 x 192^2 C=6,
16 x 256^2 C=8, 16 x 320x256 C=12; T = 80, K = 4, 8 x 8 LLR blocks, 100 outer x 5 CG)
in one plan, solved with one launch sequence per slice, with batched launches (every
slice of a shape class per launch, classes one after another, schedule autotuned) and
with those launches replayed from a HIP graph.  Same arithmetic in every mode; prints
one JSON line with slices/s per mode, the schedules and the speedups.

    python -m paper_1809_04195_amd.batching_bench [--steps 3]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=3, help="timed solves per batched mode")
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from synth import make_config

    d = make_config("mixed48_192c6_256c8_320x256c12_t80_k4")      # synthesised before the GPU is initialised (forked workers)
    import torch

    from . import (T2S_BATCHED, T2S_BATCHED_GRAPH, T2S_PER_SLICE, Plan, t2s_autotune, t2s_get_order,
                   t2s_get_schedule)

    assert torch.cuda.is_available(), "needs a GPU"
    cfg, phi, cls = d["cfg"], d["phi"], d["classes"]
    n = sum(c.nslices for c in cls)
    plan = Plan(phi, [dict(ny=c.ny, nz=c.nz, ncoils=c.ncoils, nslices=c.nslices, masks=c.masks) for c in cls],
                lam=cfg["lam"], rho=cfg["rho"], block=cfg["block"], n_outer=cfg["n_outer"], n_cg=cfg["n_cg"],
                seed=cfg["seed"])

    def load():
        for ci, c in enumerate(cls):
            plan.load(ci, 0, c.sens, c.ksp)

    def solve(mode, reps):
        times = []
        for _ in range(reps):
            load()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.reconstruct(mode)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        return min(times)

    load()
    t_tune = time.perf_counter()
    t2s_autotune(plan.handle, 2)
    t_tune = time.perf_counter() - t_tune
    res = {}
    for name, mode, reps in (("per_slice", T2S_PER_SLICE, 1), ("batched", T2S_BATCHED, args.steps),
                             ("batched_graph", T2S_BATCHED_GRAPH, args.steps)):
        solve(mode, 1)     # warm-up (graph capture, first launches)
        t = solve(mode, reps)
        res[name] = dict(s_per_batch=round(t, 4), slices_per_s=round(n / t, 2))
        print(f"[batching] {name}: {t:.3f} s for {n} slices", file=sys.stderr, flush=True)
    out = dict(workload=cfg["name"], slices=n, schedule=f"{cfg['n_outer']} outer x {cfg['n_cg']} CG",
               classes=[dict(grid=[c.ny, c.nz], coils=c.ncoils, slices=c.nslices,
                             chunk_streams=list(t2s_get_schedule(plan.handle, ci)),
                             flags=t2s_get_order(plan.handle, ci)) for ci, c in enumerate(cls)],
               autotune_s=round(t_tune, 2), **res,
               speedup_batched=round(res["per_slice"]["s_per_batch"] / res["batched"]["s_per_batch"], 2),
               speedup_graph=round(res["per_slice"]["s_per_batch"] / res["batched_graph"]["s_per_batch"], 2))
    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
