"""Launches for hardware-counter runs: the solver passes on random inputs of the two
volume workloads' shapes (HBM traffic does not depend on the values), one timed
interval each, so that `prof_summary traffic --window n` pairs the counters with the
algorithmic bytes of exactly those launches:

  window 1: 384 x 384, C = 16, T = 100, K = 5, --slots slices (default 256, the
            streaming plan of the 512-slice volume), --outer outer iterations x 5 CG
  window 2: 256 x 256, C = 8, T = 80, K = 4, 320 slices, the same schedule

with a 1 GiB device copy first (the counters' calibration).  Prints progress to stderr
and one JSON line {workload: {"kernels": {family: {launches, avg_ms,
alg_bytes_per_launch}}}}.  No worker processes (safe under rocprofv3 --pmc).

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR -o run -- \\
        python3 -m paper_1809_04195_amd.counter_bench > counter.json
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

WORKLOADS = (
    ("vol512_384x384_c16_t100_k5", 384, 384, 16, 100, 5, 0.01),
    ("vol320_256x256_c8_t80_k4", 256, 256, 8, 80, 4, 0.015),
)


def log(m):
    print(f"[counter_bench] {m}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--slots", type=int, default=256)
    ap.add_argument("--outer", type=int, default=2)
    args = ap.parse_args()
    import torch

    from . import KERNEL_NAMES, T2S_BATCHED, Plan, t2s_load_slices, t2s_profile_enable, t2s_profile_read
    from .traffic_model import alg_bytes_per_slice

    assert torch.cuda.is_available(), "needs a GPU"
    ca = torch.empty(2**28, dtype=torch.float32, device="cuda")
    cb = torch.empty_like(ca)
    cb.copy_(ca)
    torch.cuda.synchronize()
    del ca, cb
    log("copy probe: 1 GiB read + 1 GiB write")
    out = {}
    for name, ny, nz, C, Tn, K, frac in WORKLOADS:
        S = args.slots if ny == 384 else 320
        rng = np.random.default_rng(0)
        phi, _ = np.linalg.qr(rng.standard_normal((Tn, K)))
        masks = (rng.random((Tn, ny, nz)) < frac).astype(np.uint8)
        P = int(masks.sum())
        plan = Plan(phi.astype(np.float32), [dict(ny=ny, nz=nz, ncoils=C, nslices=S, masks=masks)], lam=0.01,
                    rho=0.1, n_outer=args.outer, n_cg=5, seed=1)
        g = torch.Generator(device="cuda").manual_seed(0)
        stream = torch.cuda.current_stream()
        for s0 in range(0, S, 32):
            n = min(32, S - s0)
            sens = torch.randn((n, C, ny, nz), dtype=torch.complex64, device="cuda", generator=g)
            sens /= sens.abs().square().sum(1, keepdim=True).sqrt()
            ksp = torch.randn((n, C, P), dtype=torch.complex64, device="cuda", generator=g)
            t2s_load_slices(plan.handle, 0, s0, n, sens, ksp, stream)
        torch.cuda.synchronize()
        log(f"{name}: {S} slices loaded, schedule flags {plan_order(plan)}")
        t2s_profile_enable(plan.handle, True)
        t0 = time.perf_counter()
        plan.reconstruct(T2S_BATCHED)
        torch.cuda.synchronize()
        log(f"{name}: {args.outer} outer iterations in {time.perf_counter() - t0:.2f} s")
        kern = {}
        for k, fam in enumerate(KERNEL_NAMES[:4]):
            n, ms = t2s_profile_read(plan.handle, k)
            per = alg_bytes_per_slice(fam, ny, nz, C, K, 5)
            kern[fam] = dict(launches=n, avg_ms=round(ms / max(n, 1), 4), alg_bytes_per_launch=int(per * S))
        t2s_profile_enable(plan.handle, False)
        out[name] = dict(slices=S, outer=args.outer, flags=plan_order(plan), kernels=kern)
        plan.close()
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def plan_order(plan):
    from . import t2s_get_order
    return t2s_get_order(plan.handle, 0)


if __name__ == "__main__":
    main()
