"""Write the FP64 oracle's solutions of sampled slices of the four workloads at
their own schedules (test infrastructure: calls only ``oracle/``; the inputs come
from the seeded generators of ``synth/``).

Each case runs ``oracle.t2s.admm`` on one slice exactly as the workload
prescribes and stores, in ``tests/golden/oracle_<case>.npz``:

  alpha        complex64 [K, ny, nz]   the oracle's alpha, rounded to complex64
  k_freeze     int                     outer index whose shift was frozen (-1: never)
  n_outer      int                     outer iterations run
  residuals    float64 [n_outer]       max(r_p, r_d) after every outer iteration
  cfg, cls, slice, g                   workload name, shape class, slice index in
                                       the class, global slice index of the shifts

Cases (the GPU tests run the whole plan and compare these slices):

  vol320_s{0,160,250}    320-slice 256^2 C8 T80 K4 volume, 100 outer x 5 CG
  mixed48_c{0,1,2}       mixed 48-slice batch, one slice per shape class, 100 x 5
  eval320_s{120,200}     held-out 320-slice 256^2 volume, cold start, tolerance 1e-4
  vol512_s{200,330}      512-slice 384^2 C16 T100 K5 volume, cold start, tolerance 1e-4

The tolerance cases take 0.5-1.5 h of one core each (the 384^2 ones); the
script runs the cases in parallel worker processes and skips cases whose file
already exists, so it can be resumed.

    python tests/golden/make_oracle_fixtures.py [--jobs 8] [--only vol512_s200,...]
"""

from __future__ import annotations

import argparse
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))

# (case name, workload, shape class, slice index inside the class)
CASES = [
    ("vol512_s200", "vol512_384x384_c16_t100_k5", 0, 200),
    ("vol512_s330", "vol512_384x384_c16_t100_k5", 0, 330),
    ("eval320_s120", "warmstart_eval320_256x256_c8_t80_k4", 0, 120),
    ("eval320_s200", "warmstart_eval320_256x256_c8_t80_k4", 0, 200),
    ("vol320_s0", "vol320_256x256_c8_t80_k4", 0, 0),
    ("vol320_s160", "vol320_256x256_c8_t80_k4", 0, 160),
    ("vol320_s250", "vol320_256x256_c8_t80_k4", 0, 250),
    ("mixed48_c0", "mixed48_192c6_256c8_320x256c12_t80_k4", 0, 0),
    ("mixed48_c1", "mixed48_192c6_256c8_320x256c12_t80_k4", 1, 8),
    ("mixed48_c2", "mixed48_192c6_256c8_320x256c12_t80_k4", 2, 15),
]

# Tolerance-mode decision constants of the workloads (freeze window, stall fraction,
# decision interval), the same numbers the GPU tests pass to the library.
FREEZE_WINDOW, FREEZE_STALL, CHECK_EVERY = 5, 0.05, 5


def fixture_path(case):
    return os.path.join(HERE, f"oracle_{case}.npz")


def case_inputs(workload, cls, s):
    """(cfg, phi, masks, sens, ksp, g) of slice s of class cls of workload workload."""
    import numpy as np
    from synth import CONFIGS, make_config
    cfg = CONFIGS[workload]
    if len(cfg["classes"]) == 1:
        d = make_config(workload, slices=[s], workers=1)
        g = s
    else:
        d = make_config(workload, workers=1)
        g = sum(c["nslices"] for c in cfg["classes"][:cls]) + s
    cl = d["classes"][cls]
    i = 0 if len(cfg["classes"]) == 1 else s
    return d["cfg"], d["phi"], cl.masks.astype(bool), np.ascontiguousarray(cl.sens[i]), \
        np.ascontiguousarray(cl.ksp[i]), g


def run_case(case):
    name, workload, cls, s = case
    os.environ.update(OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    sys.path.insert(0, ROOT)
    import numpy as np
    from oracle import t2s as O
    t0 = time.perf_counter()
    cfg, phi, masks, sens, ksp, g = case_inputs(workload, cls, s)
    r = O.admm(ksp, sens, phi, masks, cfg["lam"], cfg["rho"], cfg["block"], cfg["n_outer"], cfg["n_cg"],
               cfg["seed"], g=g, tol=cfg["tol"], freeze_window=FREEZE_WINDOW, freeze_stall=FREEZE_STALL,
               check_every=CHECK_EVERY)
    res = np.array([h["res"] for h in r.history])
    np.savez_compressed(fixture_path(name), alpha=r.alpha.astype(np.complex64),
                        k_freeze=r.k_freeze, n_outer=r.n_outer, residuals=res, cfg=workload, cls=cls, slice=s, g=g)
    return name, r.k_freeze, r.n_outer, time.perf_counter() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--only", type=str, default="")
    args = ap.parse_args()
    only = set(x for x in args.only.split(",") if x)
    todo = [c for c in CASES if (not only or c[0] in only) and not os.path.exists(fixture_path(c[0]))]
    print(f"{len(todo)} cases to run: {[c[0] for c in todo]}", flush=True)
    with mp.get_context("spawn").Pool(max(1, min(args.jobs, len(todo)))) as pool:
        for name, kf, n, sec in pool.imap_unordered(run_case, todo):
            print(f"{name}: k_freeze {kf}, n_outer {n}, {sec:.0f} s", flush=True)


if __name__ == "__main__":
    main()
