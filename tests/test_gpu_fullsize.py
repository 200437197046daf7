"""Parity at the workloads' full sizes.

Every slice of the volume (or mixed batch) runs in one plan, in the launch
configuration of the timed runs (all slices of a class per launch; the mixed batch
autotuned and replayed as a HIP graph).  Sampled slices are then compared with the
FP64 oracle one by one.  In the fixed-iteration mode the first n outer iterations
of a run are exactly a run stopped at n (same shifts, same CG steps), so the oracle
checks a prefix of the schedule that it can finish in seconds.  Bar: 1e-4 relative
L2 on the subspace coefficients.
"""

import sys
import time

import pytest

import paper_1809_04195_amd as T
from gpu_helpers import rel
from cpu_pool import admm_many, make_config_spawned

pytestmark = pytest.mark.gpu


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


def _jobs(cfg, phi, items, n_outer):
    """items: (class SliceSet, slice index in class, global slice index)."""
    out = []
    for cl, s, g in items:
        out.append((cl.ksp[s], cl.sens[s], phi, cl.masks.astype(bool),
                    dict(lam=cfg["lam"], rho=cfg["rho"], b=cfg["block"], n_outer=n_outer, n_cg=cfg["n_cg"],
                         seed=cfg["seed"], g=g)))
    return out


def test_vol320_sampled_slices():
    n_check = 3
    t0 = time.perf_counter()
    d = make_config_spawned(1)
    cfg, phi, cl = d["cfg"], d["phi"], d["classes"][0]
    S = cl.nslices
    _say(f"320-slice 256x256 C8 T80 K4 volume generated in {time.perf_counter() - t0:.1f} s; "
         f"{n_check} outer x {cfg['n_cg']} CG on all {S} slices, one launch per pass")
    plan = T.Plan(phi, [dict(ny=cl.ny, nz=cl.nz, ncoils=cl.ncoils, nslices=S, masks=cl.masks)], lam=cfg["lam"],
                  rho=cfg["rho"], block=cfg["block"], n_outer=n_check, n_cg=cfg["n_cg"], seed=cfg["seed"])
    T.t2s_set_schedule(plan.handle, 0, 0, 1)
    plan.load(0, 0, cl.sens, cl.ksp)
    plan.reconstruct(T.T2S_BATCHED)
    pick = [0, S // 2 + 1, S - 1]
    got = {s: plan.read(0, s, 1)[0] for s in pick}
    plan.close()
    del plan
    _free()
    refs = admm_many(_jobs(cfg, phi, [(cl, s, s) for s in pick], n_check))
    for s, ref in zip(pick, refs):
        e = rel(got[s], ref)
        _say(f"  slice {s}: rel L2 {e:.3e}")
        assert e < 1e-4, (s, e)


def test_mixed48_sampled_slices_graph_autotuned():
    n_check = 3
    t0 = time.perf_counter()
    d = make_config_spawned(2)
    cfg, phi, cls = d["cfg"], d["phi"], d["classes"]
    _say(f"mixed 48-slice batch generated in {time.perf_counter() - t0:.1f} s; autotuned, graph replay, "
         f"{n_check} outer")
    plan = T.Plan(phi, [dict(ny=c.ny, nz=c.nz, ncoils=c.ncoils, nslices=c.nslices, masks=c.masks) for c in cls],
                  lam=cfg["lam"], rho=cfg["rho"], block=cfg["block"], n_outer=n_check, n_cg=cfg["n_cg"],
                  seed=cfg["seed"])
    for ci, c in enumerate(cls):
        plan.load(ci, 0, c.sens, c.ksp)
    T.t2s_autotune(plan.handle, 2)
    for ci, c in enumerate(cls):
        plan.load(ci, 0, c.sens, c.ksp)
    plan.reconstruct(T.T2S_BATCHED_GRAPH)
    items, got, g0 = [], [], 0
    for ci, c in enumerate(cls):
        s = [0, c.nslices // 2, c.nslices - 1][ci]
        items.append((c, s, g0 + s))
        got.append(plan.read(ci, s, 1)[0])
        _say(f"  class {ci} ({c.ny}x{c.nz} C{c.ncoils}): schedule {T.t2s_get_schedule(plan.handle, ci)}")
        g0 += c.nslices
    plan.close()
    del plan
    _free()
    refs = admm_many(_jobs(cfg, phi, items, n_check))
    for (c, s, g), a, ref in zip(items, got, refs):
        e = rel(a, ref)
        _say(f"  {c.ny}x{c.nz} slice {s}: rel L2 {e:.3e}")
        assert e < 1e-4, (c.ny, c.nz, s, e)


def test_vol512_384x384_c16_k5_sampled_slices():
    """The 512-slice 384x384 volume (C=16, T=100, K=5): the full plan (all 512 slices,
    84 GB of workspace) runs.  Two readout positions inside the object are synthesised
    and placed at the first and last plan positions; the other slices carry copies of
    them, except plan position 1, which gets all-zero data (an empty slice: the
    solution is exactly zero)."""
    import torch
    n_check = 2
    S = 512
    readout = [200, 330]
    pick = [0, S - 1]
    t0 = time.perf_counter()
    d = make_config_spawned(4, slices=readout)
    cfg, phi, cl = d["cfg"], d["phi"], d["classes"][0]
    _say(f"384x384 C16 T100 K5: readout slices {readout} generated in {time.perf_counter() - t0:.1f} s; "
         f"{S}-slice plan, {n_check} outer")
    plan = T.Plan(phi, [dict(ny=cl.ny, nz=cl.nz, ncoils=cl.ncoils, nslices=S, masks=cl.masks)], lam=cfg["lam"],
                  rho=cfg["rho"], block=cfg["block"], n_outer=n_check, n_cg=cfg["n_cg"], seed=cfg["seed"])
    _say(f"  workspace {plan.nbytes / 2**30:.1f} GiB")
    sens_d = torch.from_numpy(cl.sens).cuda()
    ksp_d = torch.from_numpy(cl.ksp).cuda()
    chunk = 32
    for first in range(0, S, chunk):
        idx = torch.arange(first, min(S, first + chunk), device="cuda") % len(readout)
        plan.load(0, first, sens_d[idx].contiguous(), ksp_d[idx].contiguous())
    for i, s in enumerate(pick):
        plan.load(0, s, sens_d[i:i + 1], ksp_d[i:i + 1])
    plan.load(0, 1, sens_d[:1], torch.zeros_like(ksp_d[:1]))
    torch.cuda.synchronize()
    del sens_d, ksp_d
    plan.reconstruct(T.T2S_BATCHED)
    got = [plan.read(0, s, 1)[0] for s in pick]
    empty = plan.read(0, 1, 1)[0]
    plan.close()
    del plan
    _free()
    assert not empty.any(), "all-zero data must give an all-zero solution"
    refs = admm_many(_jobs(cfg, phi, [(cl, i, s) for i, s in enumerate(pick)], n_check))
    for s, a, ref in zip(pick, got, refs):
        e = rel(a, ref)
        _say(f"  plan slice {s}: rel L2 {e:.3e} (|ref| {abs(ref).max():.3e})")
        assert abs(ref).max() > 0
        assert e < 1e-4, (s, e)
