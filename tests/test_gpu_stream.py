"""Continuous batching (t2s_stream_*): slices streamed through fewer slots than there are
slices, each slot refilled at the stop decision of the slice it held, must give every
slice the result and the stop / freeze decisions of a batch solve of the same slices
(its own outer counter from 0, its own global index in the shift schedule).

* 13 slices of 64 x 64 (C=4, T=16, K=3, random 2D phantoms at SNR ~ U[15, 40], one
  mask set at 4 % per echo), tolerance 1e-3, through 4 slots, against one 13-slice
  batch: coefficients bitwise equal, reports equal; run in steps of at least 3
  completed slices; the same slices submitted a second time, and a third time as one
  queue entry per slice in reverse order, give the same results;
* the same with a network warm start (3-level network with random weights) against
  set_initial(net(b0)) + reconstruct;
* the held-out 320-slice 256^2 volume (C=8, T=80, K=4) to tolerance 1e-4, cold,
  through 64 slots: slices 120 and 200 against the stored FP64 oracle solutions
  (decisions exact, 1e-4 relative L2).
"""

import os
import sys
import time

import numpy as np
import pytest

import paper_1809_04195_amd as T
from gpu_helpers import rel

pytestmark = pytest.mark.gpu

NY = NZ = 64
C, NT, K = 4, 16, 3
NS, SLOTS = 13, 4
TOL_KW = dict(freeze_window=5, freeze_stall=0.05, check_every=5)
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def small(gpu):
    from synth import basis, make_training_chunk, training_masks
    phi = basis(NT, K)
    masks = training_masks(31, 1, NY, NZ, NT, 0.04, workers=1)
    sens, ksp, ptot, _ = make_training_chunk(0, NS, 31, masks, C=C, workers=1)
    assert (ptot == ptot[0]).all() and ksp.shape[2] == ptot[0]
    return phi, masks[0], np.ascontiguousarray(sens), np.ascontiguousarray(ksp)


def _plan(phi, masks, S, n_outer=200, tol=1e-3):
    return T.Plan(phi, [dict(ny=NY, nz=NZ, ncoils=C, nslices=S, masks=masks)], lam=0.01, rho=0.1, block=8,
                  n_outer=n_outer, n_cg=5, tol=tol, seed=7, **TOL_KW)


def _batch(phi, masks, sens, ksp, net=None):
    import torch
    plan = _plan(phi, masks, NS)
    plan.load(0, 0, sens, ksp)
    if net is not None:
        b0 = plan.read(0, 0, NS, T.T2S_ADJOINT, device=True)
        a0 = torch.empty_like(b0)
        for i in range(0, NS, net.max_batch):
            net.forward(b0[i:i + net.max_batch], a0[i:i + net.max_batch])
        plan.set_initial(0, 0, a0)
    code = plan.reconstruct(T.T2S_BATCHED_GRAPH)
    torch.cuda.synchronize()
    alpha = plan.read(0, 0, NS)
    reps = [plan.report(0, s) for s in range(NS)]
    plan.close()
    return code, alpha, reps


def _same_reports(got, ref):
    for s, (g, r) in enumerate(zip(got, ref)):
        assert (g["outer_iterations"], g["k_freeze"], g["converged"]) == \
            (r["outer_iterations"], r["k_freeze"], r["converged"]), (s, g, r)
        assert abs(g["r_primal"] - r["r_primal"]) <= 1e-12 * max(1.0, r["r_primal"]), (s, g, r)


def test_stream_matches_batch_cold(small):
    import torch
    phi, masks, sens, ksp = small
    code_b, alpha_b, rep_b = _batch(phi, masks, sens, ksp)
    its = [r["outer_iterations"] for r in rep_b]
    _say(f"batch of {NS}: outer iterations {its}, freezes {[r['k_freeze'] for r in rep_b]}")
    assert len(set(its)) > 2, "slices should stop at different outer iterations"
    plan = _plan(phi, masks, SLOTS)
    ds, dk = torch.from_numpy(sens).cuda(), torch.from_numpy(ksp).cuda()
    out1 = torch.zeros((NS, K, NY, NZ), dtype=torch.complex64, device="cuda")
    out2 = torch.zeros_like(out1)
    out3 = torch.zeros_like(out1)
    plan.stream_open(None, T.T2S_BATCHED_GRAPH)
    rep1 = plan.stream_submit(ds, dk, out1, 0)
    rep2 = plan.stream_submit(ds, dk, out2, 0)      # the same slices again
    # and once more, one queue entry per slice in reverse order (refills across entries)
    rep3 = [plan.stream_submit(ds[g:g + 1], dk[g:g + 1], out3[g:g + 1], g) for g in reversed(range(NS))]
    steps, prev, code = 0, 0, 0
    while True:
        c, st = plan.stream_run(3)
        code, done, inflight = max(code, c), st["done"], st["in_flight"]
        steps += 1
        assert done - prev >= 3 or inflight == 0, (done, prev, inflight)
        prev = done
        if inflight == 0:
            break
    assert st["loaded"] == 3 * NS
    assert st["slice_outer"] == 3 * sum(its)
    torch.cuda.synchronize()
    _say(f"stream through {SLOTS} slots: {done} slices in {steps} calls")
    assert done == 3 * NS and code == code_b
    rep3 = [T.Plan.stream_reports(r)[0] for r in reversed(rep3)]
    for out, rep in ((out1, T.Plan.stream_reports(rep1)), (out2, T.Plan.stream_reports(rep2)), (out3, rep3)):
        got = out.cpu().numpy()
        d = float(np.abs(got - alpha_b).max())
        _say(f"  max |alpha_stream - alpha_batch| = {d:.3e} (rel L2 {rel(got, alpha_b):.2e})")
        assert d == 0.0
        _same_reports(rep, rep_b)
    plan.stream_close()
    plan.close()


def test_stream_matches_batch_warm_start(small):
    import torch
    phi, masks, sens, ksp = small
    net = T.UNet(K, 16, 3, max_batch=SLOTS, H=NY, W=NZ)
    net.set_params(net.init_params(seed=5))
    code_b, alpha_b, rep_b = _batch(phi, masks, sens, ksp, net)
    plan = _plan(phi, masks, SLOTS)
    ds, dk = torch.from_numpy(sens).cuda(), torch.from_numpy(ksp).cuda()
    out = torch.zeros((NS, K, NY, NZ), dtype=torch.complex64, device="cuda")
    plan.stream_open(net, T.T2S_BATCHED)
    rep = plan.stream_submit(ds, dk, out, 0)
    code, st = plan.stream_run(0)
    torch.cuda.synchronize()
    assert st["done"] == NS and st["in_flight"] == 0 and code == code_b
    got = out.cpu().numpy()
    d = float(np.abs(got - alpha_b).max())
    _say(f"warm start through {SLOTS} slots: max |alpha_stream - alpha_batch| = {d:.3e}, outer iterations "
         f"{[r['outer_iterations'] for r in T.Plan.stream_reports(rep)]}")
    assert d == 0.0
    _same_reports(T.Plan.stream_reports(rep), rep_b)
    plan.stream_close()
    plan.close()
    net.close()


def test_stream_open_rejects_mismatched_network(small):
    phi, masks, _, _ = small
    plan = _plan(phi, masks, SLOTS)
    net = T.UNet(K, 16, 3, max_batch=2, H=NY, W=2 * NZ)
    with pytest.raises(T.T2SError) as e:
        plan.stream_open(net)
    assert e.value.code == T.T2S_ESHAPE
    plan.close()
    net.close()


def test_eval320_streamed_through_64_slots_against_oracle():
    import torch
    from cpu_pool import make_config_spawned
    t0 = time.perf_counter()
    d = make_config_spawned("warmstart_eval320_256x256_c8_t80_k4")
    cfg, phi, cl = d["cfg"], d["phi"], d["classes"][0]
    _say(f"held-out 320-slice 256x256 volume generated in {time.perf_counter() - t0:.1f} s; streamed through "
         f"64 slots, cold, tolerance {cfg['tol']}")
    plan = T.Plan(phi, [dict(ny=cl.ny, nz=cl.nz, ncoils=cl.ncoils, nslices=64, masks=cl.masks)], lam=cfg["lam"],
                  rho=cfg["rho"], block=cfg["block"], n_outer=cfg["n_outer"], n_cg=cfg["n_cg"], tol=cfg["tol"],
                  seed=cfg["seed"], **TOL_KW)
    ds, dk = torch.from_numpy(cl.sens).cuda(), torch.from_numpy(cl.ksp).cuda()
    out = torch.empty((cl.nslices, phi.shape[1], cl.ny, cl.nz), dtype=torch.complex64, device="cuda")
    plan.stream_open(None, T.T2S_BATCHED_GRAPH)
    rep = plan.stream_submit(ds, dk, out, 0)
    t1 = time.perf_counter()
    code, st = plan.stream_run(0)
    torch.cuda.synchronize()
    _say(f"  {st['done']} slices in {time.perf_counter() - t1:.1f} s")
    assert code == 0 and st["done"] == cl.nslices and st["in_flight"] == 0
    reps = T.Plan.stream_reports(rep)
    assert all(r["converged"] == 1 for r in reps)
    for s in (120, 200):
        with np.load(os.path.join(GOLDEN, f"oracle_eval320_s{s}.npz")) as f:
            fx = {k: f[k] for k in f.files}
        r = reps[s]
        _say(f"  slice {s}: freeze {r['k_freeze']} stop {r['outer_iterations']} (oracle {int(fx['k_freeze'])}, "
             f"{int(fx['n_outer'])})")
        assert (r["k_freeze"], r["outer_iterations"]) == (int(fx["k_freeze"]), int(fx["n_outer"]))
        e = rel(out[s].cpu().numpy(), fx["alpha"])
        _say(f"  slice {s}: rel L2 {e:.3e}")
        assert e < 1e-4
    plan.stream_close()
    plan.close()
