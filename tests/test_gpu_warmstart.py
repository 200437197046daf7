"""The learned warm start against the method without it, on a small workload trained
here from the solver's own outputs (128 x 128 slices, C=8, T=32, K=4, 2 % per echo,
one mask set, random 2D phantoms, SNR ~ U[15, 40]; 3-level network, 16 base filters).

* gain: a network trained on 1024 solver solutions (100 x 5 ADMM each) starts the
  tolerance-mode ADMM (tol 1e-4) on 16 held-out slices; it must need fewer outer
  iterations than the cold start, every slice still converging;
* fallback: a network with random weights (a bad warm start) must still reach the
  same tolerance on every slice, ending near the cold solution (the remaining
  difference comes from the block shift the stop rule freezes, which depends on the
  start).
"""

import sys

import numpy as np
import pytest

import paper_1809_04195_amd as T

pytestmark = pytest.mark.gpu

NY = NZ = 128
C, NT, K = 8, 32, 4
FRAC = 0.02
LAM, RHO, BLOCK = 0.01, 0.1, 8
SEED = 20


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def workload(gpu):
    from synth import basis, make_training_chunk, training_masks
    phi = basis(NT, K)
    masks = training_masks(SEED, 1, NY, NZ, NT, FRAC, workers=1)
    train = make_training_chunk(0, 1024, SEED, masks, C=C, workers=8)
    held = make_training_chunk(100000, 16, SEED, masks, C=C, workers=4)
    return phi, masks[0], train, held


def _plan(phi, masks, n, tol, n_outer):
    return T.Plan(phi, [dict(ny=NY, nz=NZ, ncoils=C, nslices=n, masks=masks)], lam=LAM, rho=RHO, block=BLOCK,
                  n_outer=n_outer, n_cg=5, tol=tol, seed=SEED, freeze_window=5, freeze_stall=0.05, check_every=5)


def _load(plan, data):
    sens, ksp, ptot, _ = data
    plan.load(0, 0, np.ascontiguousarray(sens), np.ascontiguousarray(ksp[:, :, :int(ptot[0])]))


def _solve_tol(phi, masks, data, net):
    """Tolerance-mode ADMM from the cold start (net None) or from net(b0)."""
    import torch
    n = data[0].shape[0]
    plan = _plan(phi, masks, n, 1e-4, 500)
    _load(plan, data)
    if net is not None:
        b0 = plan.read(0, 0, n, T.T2S_ADJOINT, device=True)
        a0 = torch.empty_like(b0)
        net.forward(b0, a0)
        plan.set_initial(0, 0, a0)
    code = plan.reconstruct(T.T2S_BATCHED_GRAPH)
    reps = [plan.report(0, s) for s in range(n)]
    alpha = plan.read(0, 0, n)
    plan.close()
    return code, reps, alpha


@pytest.fixture(scope="module")
def trained(workload):
    import torch
    phi, masks, train, _ = workload
    n = train[0].shape[0]
    plan = _plan(phi, masks, n, 0.0, 100)
    _load(plan, train)
    plan.reconstruct(T.T2S_BATCHED_GRAPH)
    b0 = plan.read(0, 0, n, T.T2S_ADJOINT, device=True)
    target = plan.read(0, 0, n, T.T2S_ALPHA, device=True)
    plan.close()
    net = T.UNet(K, 16, 3, max_batch=16, H=NY, W=NZ)
    net.set_params(net.init_params(SEED))
    rng = np.random.default_rng(SEED)
    epochs = 40
    for ep in range(epochs):
        lr = 2e-3 * 0.5 * (1 + np.cos(np.pi * ep / epochs))
        perm = torch.from_numpy(rng.permutation(n)).cuda()
        for i in range(0, n, 16):
            idx = perm[i:i + 16]
            l = net.train_step(b0[idx].contiguous(), target[idx].contiguous(), lr, want_loss=(i == 0))
            if i == 0:
                loss = l
        if ep % 10 == 0 or ep == epochs - 1:
            _say(f"  epoch {ep}: loss of the first batch {loss:.5f}")
    yield net
    net.close()


def test_trained_network_saves_outer_iterations(workload, trained):
    phi, masks, _, held = workload
    code_c, cold, a_cold = _solve_tol(phi, masks, held, None)
    code_w, warm, a_warm = _solve_tol(phi, masks, held, trained)
    ic = np.array([r["outer_iterations"] for r in cold])
    iw = np.array([r["outer_iterations"] for r in warm])
    _say(f"  outer iterations to 1e-4, cold: mean {ic.mean():.1f} {ic.tolist()}")
    _say(f"  outer iterations to 1e-4, warm: mean {iw.mean():.1f} {iw.tolist()}")
    assert code_c == 0 and code_w == 0
    assert all(r["converged"] for r in cold + warm)
    assert iw.mean() < 0.9 * ic.mean(), (iw.mean(), ic.mean())
    d = np.linalg.norm(a_warm - a_cold) / np.linalg.norm(a_cold)
    _say(f"  warm vs cold solution: rel L2 {d:.3e}")
    assert d < 5e-2


def test_random_network_still_converges(workload):
    phi, masks, _, held = workload
    net = T.UNet(K, 16, 3, max_batch=16, H=NY, W=NZ)
    p = net.init_params(123)
    p = p + 0.05 * np.random.default_rng(123).standard_normal(p.size).astype(np.float32)
    net.set_params(p)
    code_c, cold, a_cold = _solve_tol(phi, masks, held, None)
    code_r, rnd, a_rnd = _solve_tol(phi, masks, held, net)
    net.close()
    ic = np.array([r["outer_iterations"] for r in cold])
    ir = np.array([r["outer_iterations"] for r in rnd])
    d = np.linalg.norm(a_rnd - a_cold) / np.linalg.norm(a_cold)
    _say(f"  random-weights start: outer mean {ir.mean():.1f} (cold {ic.mean():.1f}); vs cold solution {d:.3e}")
    assert code_r == 0
    assert all(r["converged"] for r in rnd)
    assert max(max(r["r_primal"], r["r_dual"]) for r in rnd) <= 1e-4
    assert d < 5e-2
