"""GPU parity of the post-step (wavelet soft-threshold of the coefficient images and
back-projection onto echo times) against the FP64 oracle.  Elementwise-exact steps
in fp32: 1e-6 relative L2; after a whole ADMM run: 1e-4."""

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


def _loaded_plan(ny, nz, C, Tn, K, S, seed, **kw):
    phi, sens, masks, ksp = random_problem(seed, ny, nz, C, Tn, K, S=S, frac=0.3)
    plan = T.Plan(phi, [dict(ny=ny, nz=nz, ncoils=C, nslices=S, masks=masks)], lam=0.02, rho=0.1, seed=3, **kw)
    plan.load(0, 0, sens, ksp)
    return plan, phi, sens, masks, ksp


@pytest.mark.parametrize("ny,nz,K", [(64, 64, 3), (48, 32, 2)])
def test_wavelet_denoise_parity(ny, nz, K):
    rng = np.random.default_rng(ny + nz + K)
    plan, *_ = _loaded_plan(ny, nz, 2, 6, K, 2, ny + K)
    a0 = crandn(rng, 2, K, ny, nz)
    thr = float(0.5 * np.median(np.abs(a0)))
    for levels in (1, 2, 3, 4):
        _say(f"wavelet denoise {ny}x{nz} K{K} levels {levels} thresh {thr:.3f}")
        plan.set_initial(0, 0, a0)
        plan.wavelet_denoise(0, 1, 1, levels, thr)           # slice 1 only
        got = plan.read(0, 0, 2)
        assert np.array_equal(got[0], a0[0])
        e = rel(got[1], O.wavelet_denoise(a0[1], levels, thr))
        _say(f"  rel L2 {e:.3e}")
        assert e < 1e-6
    plan.close()


def test_backproject_parity():
    rng = np.random.default_rng(5)
    plan, phi, *_ = _loaded_plan(64, 32, 2, 12, 4, 3, 61)
    a0 = crandn(rng, 3, 4, 64, 32)
    plan.set_initial(0, 0, a0)
    sel = phi[[2, 6, 11]]
    out = plan.backproject(0, 1, 2, sel).cpu().numpy()
    for i in range(2):
        e = rel(out[i], O.backproject(a0[1 + i], sel))
        _say(f"backproject slice {1 + i}: rel L2 {e:.3e}")
        assert e < 1e-6


def test_solve_denoise_backproject_pipeline():
    _say("ADMM 6 x 4 -> Haar 3 levels -> 3 echo times, 64x64 C3 T12 K3, 2 slices")
    plan, phi, sens, masks, ksp = _loaded_plan(64, 64, 3, 12, 3, 2, 71, n_outer=6, n_cg=4)
    plan.reconstruct()
    plan.wavelet_denoise(0, 0, 2, 3, 0.05)
    sel = phi[[1, 5, 10]]
    out = plan.backproject(0, 0, 2, sel).cpu().numpy()
    plan.close()
    for s in range(2):
        ref = O.admm(ksp[s], sens[s], phi, masks.astype(bool), 0.02, 0.1, 8, 6, 4, 3, g=s)
        want = O.backproject(O.wavelet_denoise(ref.alpha, 3, 0.05), sel)
        e = rel(out[s], want)
        _say(f"  slice {s}: rel L2 {e:.3e}")
        assert e < 1e-4


def test_post_argument_errors():
    plan, phi, *_ = _loaded_plan(32, 32, 2, 6, 2, 1, 81)
    for levels, thr in ((0, 0.1), (5, 0.1), (2, float("nan")), (2, -1.0)):
        with pytest.raises(T.T2SError):
            plan.wavelet_denoise(0, 0, 1, levels, thr)
    with pytest.raises(T.T2SError):
        plan.wavelet_denoise(0, 0, 2, 2, 0.1)                 # slice range past the class
    with pytest.raises(T.T2SError):
        plan.backproject(0, 0, 1, np.zeros((9, 2)))           # more than 8 echo times
    with pytest.raises(T.T2SError):
        plan.backproject(0, 0, 1, np.full((1, 2), np.inf))
    plan.close()
