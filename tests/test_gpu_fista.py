"""GPU parity of the FISTA solver (the paper's own, Sec. II-A) and of its power-iteration
step size, through the C ABI, against the FP64 oracle.

Same bar as the ADMM runs: 1e-4 relative L2 on the subspace coefficients; the
largest eigenvalue of A^H A to 1e-4 relative.
"""

import sys

import numpy as np
import pytest

import paper_1809_04195_amd as T
from oracle import t2s as O
from gpu_helpers import crandn, random_problem, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu(gpu):
    return gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _slice64():
    from synth import make_config
    d = make_config("slice64_c4_t16_k3")
    return d["cfg"], d["phi"], d["classes"][0]


def _oracle_L(ksp, sens, phi, masks, iters):
    m = masks.astype(bool)
    b0 = O.adjoint(ksp, sens, phi, m)
    return O.lipschitz(sens, O.space_time_kernel(phi, m), b0, iters)


def test_lipschitz_parity_and_empty_slice():
    _say("power iteration: 3 slices 48x64 C3 T8 K3 (slice 2 has no data), 30 iterations")
    phi, sens, masks, ksp = random_problem(31, 48, 64, 3, 8, 3, S=3, frac=0.3)
    ksp[2] = 0
    plan = T.Plan(phi, [dict(ny=48, nz=64, ncoils=3, nslices=3, masks=masks)], lam=0.02, rho=0.1, seed=1)
    plan.load(0, 0, sens, ksp)
    L = plan.lipschitz(0, iters=30)
    plan.close()
    for s in range(2):
        ref = _oracle_L(ksp[s], sens[s], phi, masks, 30)
        _say(f"  slice {s}: L gpu {L[s]:.7f} oracle {ref:.7f}")
        assert abs(L[s] - ref) < 1e-4 * ref
    assert L[2] == 0.0


def test_fista_slice64_parity():
    cfg, phi, cl = _slice64()
    n_iter = 20
    _say(f"FISTA parity: 64x64 C4 T16 K3, {n_iter} iterations, shift schedule seed {cfg['seed']}")
    m = cl.masks.astype(bool)
    step = np.float32(0.95 / _oracle_L(cl.ksp[0], cl.sens[0], phi, cl.masks, 200))
    plan = T.Plan(phi, [dict(ny=cl.ny, nz=cl.nz, ncoils=cl.ncoils, nslices=1, masks=cl.masks)], lam=cfg["lam"],
                  rho=cfg["rho"], block=cfg["block"], n_outer=cfg["n_outer"], seed=cfg["seed"])
    plan.load(0, 0, cl.sens, cl.ksp)
    plan.fista(n_iter, float(step))
    got = plan.read(0, 0, 1)[0]
    rep = plan.report(0, 0)
    plan.close()
    ref = O.fista(cl.ksp[0], cl.sens[0], phi, m, cfg["lam"], cfg["block"], n_iter, step=float(step),
                  seed=cfg["seed"], g=0)
    prev = O.fista(cl.ksp[0], cl.sens[0], phi, m, cfg["lam"], cfg["block"], n_iter - 1, step=float(step),
                   seed=cfg["seed"], g=0)
    e = rel(got, ref)
    _say(f"  rel L2 alpha {e:.3e}")
    assert e < 1e-4
    # report: relative size of the last step
    b0n = np.linalg.norm(O.adjoint(cl.ksp[0], cl.sens[0], phi, m))
    d = max(np.linalg.norm(ref), np.linalg.norm(prev), 0.01 * b0n)
    want = np.linalg.norm(ref - prev) / d
    _say(f"  last relative step gpu {rep['r_primal']:.4e} oracle {want:.4e}")
    assert rep["outer_iterations"] == n_iter
    assert abs(rep["r_primal"] - want) <= 2e-2 * want
    assert rep["r_dual"] == 0.0


def test_fista_multiclass_batched_and_per_slice():
    _say("FISTA: two shape classes (64x64 C4, 32x48 C2), 2 slices each, 12 iterations, batched vs per-slice")
    phi, sA, mA, kA = random_problem(41, 64, 64, 4, 8, 3, S=2, frac=0.25)
    _, sB, mB, kB = random_problem(42, 32, 48, 2, 8, 3, S=2, frac=0.25)
    classes = [dict(ny=64, nz=64, ncoils=4, nslices=2, masks=mA), dict(ny=32, nz=48, ncoils=2, nslices=2, masks=mB)]
    step, lam, seed, n_iter = 0.9, 0.05, 6, 12
    outs = []
    for mode in (T.T2S_BATCHED, T.T2S_PER_SLICE):
        plan = T.Plan(phi, classes, lam=lam, rho=0.1, n_outer=20, seed=seed)
        plan.load(0, 0, sA, kA)
        plan.load(1, 0, sB, kB)
        plan.fista(n_iter, step, mode=mode)
        outs.append([plan.read(0, 0, 2), plan.read(1, 0, 2)])
        plan.close()
    for ci in range(2):
        assert np.array_equal(outs[0][ci], outs[1][ci])
    for ci, (sens, masks, ksp) in enumerate([(sA, mA, kA), (sB, mB, kB)]):
        for s in range(2):
            ref = O.fista(ksp[s], sens[s], phi, masks.astype(bool), lam, 8, n_iter, step=step, seed=seed,
                          g=ci * 2 + s)
            e = rel(outs[0][ci][s], ref)
            _say(f"  class {ci} slice {s}: rel L2 {e:.3e}")
            assert e < 1e-4, (ci, s, e)


@pytest.mark.parametrize("ny,nz,C,Tn,K", [(320, 16, 2, 6, 4), (96, 32, 2, 6, 5)])
def test_fista_ragged_and_k5(ny, nz, C, Tn, K):
    _say(f"FISTA parity ny={ny} nz={nz} C={C} T={Tn} K={K}, 8 iterations, 2 slices")
    phi, sens, masks, ksp = random_problem(ny + nz + 7 * K, ny, nz, C, Tn, K, S=2, frac=0.3)
    plan = T.Plan(phi, [dict(ny=ny, nz=nz, ncoils=C, nslices=2, masks=masks)], lam=0.03, rho=0.1, n_outer=10,
                  seed=2)
    plan.load(0, 0, sens, ksp)
    plan.fista(8, 0.8)
    got = plan.read(0, 0, 2)
    plan.close()
    for s in range(2):
        ref = O.fista(ksp[s], sens[s], phi, masks.astype(bool), 0.03, 8, 8, step=0.8, seed=2, g=s)
        e = rel(got[s], ref)
        _say(f"  slice {s}: rel L2 {e:.3e}")
        assert e < 1e-4, (s, e)


def test_fista_warm_start_and_continuation():
    _say("FISTA from a set_initial start, then a second call continuing from its result (64x64 C4 K3)")
    cfg, phi, cl = _slice64()
    m = cl.masks.astype(bool)
    rng = np.random.default_rng(8)
    b0 = O.adjoint(cl.ksp[0], cl.sens[0], phi, m)
    a0 = (b0 + 0.01 * crandn(rng, *b0.shape)).astype(np.complex64)
    plan = T.Plan(phi, [dict(ny=cl.ny, nz=cl.nz, ncoils=cl.ncoils, nslices=1, masks=cl.masks)], lam=cfg["lam"],
                  rho=cfg["rho"], n_outer=20, seed=cfg["seed"])
    plan.load(0, 0, cl.sens, cl.ksp)
    plan.set_initial(0, 0, a0[None])
    plan.fista(6, 0.9)
    got1 = plan.read(0, 0, 1)[0]
    plan.fista(4, 0.9)
    got2 = plan.read(0, 0, 1)[0]
    plan.close()
    ref1 = O.fista(cl.ksp[0], cl.sens[0], phi, m, cfg["lam"], 8, 6, step=0.9, seed=cfg["seed"], g=0, alpha0=a0)
    # a new call restarts the momentum and the shift schedule from its own start
    ref2 = O.fista(cl.ksp[0], cl.sens[0], phi, m, cfg["lam"], 8, 4, step=0.9, seed=cfg["seed"], g=0,
                   alpha0=got1.astype(np.complex128))
    e1, e2 = rel(got1, ref1), rel(got2, ref2)
    _say(f"  rel L2 after 6 {e1:.3e}, after 6 + 4 {e2:.3e}")
    assert e1 < 1e-4 and e2 < 1e-4


def test_fista_argument_errors():
    cfg, phi, cl = _slice64()
    plan = T.Plan(phi, [dict(ny=cl.ny, nz=cl.nz, ncoils=cl.ncoils, nslices=1, masks=cl.masks)], lam=0.01, rho=0.1,
                  seed=0)
    with pytest.raises(T.T2SError):
        plan.fista(3, 0.5)                      # nothing loaded yet
    plan.load(0, 0, cl.sens, cl.ksp)
    for n_iter, step, mode in ((-1, 0.5, T.T2S_BATCHED), (3, 0.0, T.T2S_BATCHED), (3, float("nan"), T.T2S_BATCHED),
                               (3, 0.5, T.T2S_BATCHED_GRAPH)):
        with pytest.raises(T.T2SError):
            plan.fista(n_iter, step, mode=mode)
    with pytest.raises(T.T2SError):
        plan.lipschitz(0, iters=0)
    plan.close()
