"""Parity at the workloads' full sizes and their own schedules.

Every slice of the volume (or mixed batch) runs in one plan, in the launch
configuration of the timed runs (all slices of a class per launch, one outer
iteration replayed from a HIP graph; the mixed batch autotuned).  Sampled slices
are compared one by one with the FP64 oracle's solution of the same slice at the
same schedule, stored in tests/golden/oracle_*.npz by
tests/golden/make_oracle_fixtures.py (which calls only the oracle, on the same
seeded inputs):

* 320-slice 256^2 volume, 100 outer x 5 CG: slices 0 (edge), 160, 250;
* mixed 48-slice batch, 100 x 5: one slice per shape class;
* held-out 320-slice 256^2 volume, cold start to tolerance 1e-4: slices 120, 200,
  whose stop-rule decisions (freeze index, outer iterations) must be the oracle's;
* 512-slice 384^2 C16 T100 K5 volume to tolerance 1e-4: readout slices 200, 330.

Bar: 1e-4 relative L2 on the subspace coefficients.  The 320-slice run also checks
the drift of the CG residual, which the library updates incrementally across the
whole run instead of recomputing it.
"""

import os
import sys
import time

import numpy as np
import pytest

import paper_1809_04195_amd as T
from gpu_helpers import rel
from cpu_pool import make_config_spawned

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL_KW = dict(freeze_window=5, freeze_stall=0.05, check_every=5)


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu(gpu):
    return gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _free():
    import torch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _fixture(case):
    path = os.path.join(GOLDEN, f"oracle_{case}.npz")
    assert os.path.exists(path), f"{path} is missing: run tests/golden/make_oracle_fixtures.py"
    with np.load(path) as f:
        return {k: f[k] for k in f.files}


def _plan(cfg, phi, classes, nslices=None, tol=None):
    tol = cfg["tol"] if tol is None else tol
    return T.Plan(phi, [dict(ny=c.ny, nz=c.nz, ncoils=c.ncoils, nslices=nslices or c.nslices, masks=c.masks)
                        for c in classes], lam=cfg["lam"], rho=cfg["rho"], block=cfg["block"],
                  n_outer=cfg["n_outer"], n_cg=cfg["n_cg"], tol=tol, seed=cfg["seed"], **TOL_KW)


def _compare(tag, got, fx):
    e = rel(got, fx["alpha"])
    per_k = [rel(got[k], fx["alpha"][k]) for k in range(got.shape[0])]
    _say(f"  {tag}: rel L2 {e:.3e} (per coefficient {', '.join(f'{x:.1e}' for x in per_k)})")
    assert np.abs(fx["alpha"]).max() > 0
    assert e < 1e-4, (tag, e)


def test_vol320_full_schedule_and_cg_residual_drift():
    import torch
    t0 = time.perf_counter()
    d = make_config_spawned("vol320_256x256_c8_t80_k4")
    cfg, phi, cl = d["cfg"], d["phi"], d["classes"][0]
    _say(f"320-slice 256x256 C8 T80 K4 volume generated in {time.perf_counter() - t0:.1f} s; "
         f"{cfg['n_outer']} outer x {cfg['n_cg']} CG, batched graph")
    plan = _plan(cfg, phi, [cl])
    plan.load(0, 0, cl.sens, cl.ksp)
    plan.reconstruct(T.T2S_BATCHED_GRAPH)
    torch.cuda.synchronize()
    for s in (0, 160, 250):
        _compare(f"slice {s}", plan.read(0, s, 1)[0], _fixture(f"vol320_s{s}"))
    # CG residual tracked over 100 x 5 steps vs recomputed: r = b0 + rho (z - u) - (A^H A + rho) alpha
    s = 160
    al = plan.read(0, s, 1, T.T2S_ALPHA, device=True)
    z = plan.read(0, s, 1, T.T2S_Z, device=True)
    u = plan.read(0, s, 1, T.T2S_U, device=True)
    b0 = plan.read(0, s, 1, T.T2S_ADJOINT, device=True)
    r = plan.read(0, s, 1, T.T2S_RESIDUAL, device=True)
    ma = torch.empty_like(al)
    T.t2s_apply_normal(plan.handle, 0, s, 1, al, ma, cfg["rho"])
    r_exp = b0 + cfg["rho"] * (z - u) - ma
    drift = float(torch.linalg.vector_norm(r - r_exp) / torch.linalg.vector_norm(b0))
    size = float(torch.linalg.vector_norm(r_exp) / torch.linalg.vector_norm(b0))
    _say(f"  CG residual after 100 outer x 5 CG: ||r_tracked - r_recomputed|| / ||b0|| = {drift:.3e} "
         f"(||r|| / ||b0|| = {size:.3e})")
    plan.close()
    del plan
    _free()
    assert drift < 1e-4, drift


def test_mixed48_full_schedule_graph_autotuned():
    t0 = time.perf_counter()
    d = make_config_spawned("mixed48_192c6_256c8_320x256c12_t80_k4")
    cfg, phi, cls = d["cfg"], d["phi"], d["classes"]
    _say(f"mixed 48-slice batch generated in {time.perf_counter() - t0:.1f} s; autotuned, graph replay, "
         f"{cfg['n_outer']} x {cfg['n_cg']}")
    plan = _plan(cfg, phi, cls)
    for ci, c in enumerate(cls):
        plan.load(ci, 0, c.sens, c.ksp)
    T.t2s_autotune(plan.handle, 2)
    for ci, c in enumerate(cls):
        plan.load(ci, 0, c.sens, c.ksp)
    plan.reconstruct(T.T2S_BATCHED_GRAPH)
    for ci, c in enumerate(cls):
        fx = _fixture(f"mixed48_c{ci}")
        assert int(fx["cls"]) == ci
        s = int(fx["slice"])
        _say(f"  class {ci} ({c.ny}x{c.nz} C{c.ncoils}): schedule {T.t2s_get_schedule(plan.handle, ci)}")
        _compare(f"{c.ny}x{c.nz} slice {s}", plan.read(ci, s, 1)[0], fx)
    plan.close()
    del plan
    _free()


def _check_tolerance_slice(plan, s, fx, tag):
    rep = plan.report(0, s)
    _say(f"  {tag}: GPU freeze {rep['k_freeze']} stop {rep['outer_iterations']}, oracle freeze "
         f"{int(fx['k_freeze'])} stop {int(fx['n_outer'])}; final residual {max(rep['r_primal'], rep['r_dual']):.2e}")
    assert rep["converged"] == 1
    assert rep["k_freeze"] == int(fx["k_freeze"]) and rep["outer_iterations"] == int(fx["n_outer"]), (tag, rep)
    _compare(tag, plan.read(0, s, 1)[0], fx)


def test_eval320_tolerance_mode():
    t0 = time.perf_counter()
    d = make_config_spawned("warmstart_eval320_256x256_c8_t80_k4")
    cfg, phi, cl = d["cfg"], d["phi"], d["classes"][0]
    _say(f"held-out 320-slice 256x256 volume generated in {time.perf_counter() - t0:.1f} s; cold start to "
         f"tolerance {cfg['tol']}, batched graph")
    plan = _plan(cfg, phi, [cl])
    plan.load(0, 0, cl.sens, cl.ksp)
    code = plan.reconstruct(T.T2S_BATCHED_GRAPH)
    assert code == 0
    for s in (120, 200):
        _check_tolerance_slice(plan, s, _fixture(f"eval320_s{s}"), f"slice {s}")
    plan.close()
    del plan
    _free()


def test_vol512_384x384_c16_k5_tolerance_mode():
    """The 512-slice 384x384 volume (C=16, T=100, K=5) plan, 84 GB of workspace.
    Readout slices 200 and 330 are synthesised and placed at their own positions; every
    8th other position carries a copy of one of them (its own shifts, so its own
    trajectory) and the rest all-zero data (no signal: solution exactly zero, stopped at
    the first decision)."""
    import torch
    S = 512
    readout = [200, 330]
    t0 = time.perf_counter()
    d = make_config_spawned("vol512_384x384_c16_t100_k5", slices=readout)
    cfg, phi, cl = d["cfg"], d["phi"], d["classes"][0]
    _say(f"384x384 C16 T100 K5: readout slices {readout} generated in {time.perf_counter() - t0:.1f} s; "
         f"{S}-slice plan to tolerance {cfg['tol']}, batched graph")
    plan = _plan(cfg, phi, [cl], nslices=S)
    _say(f"  workspace {plan.nbytes / 2**30:.1f} GiB")
    sens_d = torch.from_numpy(cl.sens).cuda()
    ksp_d = torch.from_numpy(cl.ksp).cuda()
    zeros = torch.zeros_like(ksp_d[:1])
    for p in range(S):
        if p in readout:
            i = readout.index(p)
            plan.load(0, p, sens_d[i:i + 1], ksp_d[i:i + 1])
        elif p % 8 == 0:
            plan.load(0, p, sens_d[(p // 8) % 2:(p // 8) % 2 + 1], ksp_d[(p // 8) % 2:(p // 8) % 2 + 1])
        else:
            plan.load(0, p, sens_d[:1], zeros)
    torch.cuda.synchronize()
    del sens_d, ksp_d
    t1 = time.perf_counter()
    code = plan.reconstruct(T.T2S_BATCHED_GRAPH)
    torch.cuda.synchronize()
    _say(f"  solved in {time.perf_counter() - t1:.1f} s")
    assert code == 0
    for s in readout:
        _check_tolerance_slice(plan, s, _fixture(f"vol512_s{s}"), f"plan slice {s}")
    empty = plan.read(0, 1, 1)[0]
    rep = plan.report(0, 1)
    plan.close()
    del plan
    _free()
    assert not empty.any(), "all-zero data must give an all-zero solution"
    assert rep["outer_iterations"] == TOL_KW["check_every"] and rep["converged"] == 1
