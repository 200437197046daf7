"""GPU parity of the readout pre-step (the 1D inverse DFT that decouples a 3D
acquisition into slices) and of a whole volume fed from 3D data, against the FP64
oracle.  Single transforms: 1e-6 relative L2; whole ADMM runs: 1e-4."""

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


@pytest.mark.parametrize("nx,C,P", [(64, 3, 1001), (320, 2, 777), (16, 1, 5), (512, 2, 403), (192, 4, 0)])
def test_readout_ifft_parity(nx, C, P):
    import torch
    _say(f"readout pre-step nx={nx} C={C} P={P}")
    rng = np.random.default_rng(nx + P)
    k = crandn(rng, C, P, nx)
    dk = torch.from_numpy(k).cuda()
    out = torch.full((nx, C, P), float("nan"), dtype=torch.complex64, device="cuda")
    T.t2s_readout_ifft(dk, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    if P == 0:
        return
    ref = O.readout_ifft(k)
    e = rel(got, ref)
    _say(f"  rel L2 {e:.3e}")
    assert np.all(np.isfinite(got)) and e < 1e-6


def test_volume_from_3d_data_parity():
    import torch
    nx, ny, nz, C, Tn, K = 32, 32, 32, 2, 6, 2
    _say(f"volume from 3D data: readout {nx}, slices {ny}x{nz} C{C} T{Tn} K{K}, 4 outer x 3 CG")
    phi, sens, masks, _ = random_problem(51, ny, nz, C, Tn, K, S=nx, frac=0.3)
    rng = np.random.default_rng(52)
    P = int(masks.sum())
    k3 = crandn(rng, C, P, nx)                      # 3D samples: coil, (echo, y, z) entry, kx
    dk3 = torch.from_numpy(k3).cuda()
    dksp = torch.empty((nx, C, P), dtype=torch.complex64, device="cuda")
    T.t2s_readout_ifft(dk3, dksp)
    dsens = torch.from_numpy(sens).cuda()
    plan = T.Plan(phi, [dict(ny=ny, nz=nz, ncoils=C, nslices=nx, masks=masks)], lam=0.02, rho=0.1, n_outer=4,
                  n_cg=3, seed=7)
    stream = torch.cuda.current_stream()
    T.t2s_load_slices(plan.handle, 0, 0, nx, dsens, dksp, stream)
    plan.reconstruct()
    got = plan.read(0, 0, nx)
    plan.close()
    y = O.readout_ifft(k3)
    for x in (0, 13, nx - 1):
        ref = O.admm(y[x], sens[x], phi, masks.astype(bool), 0.02, 0.1, 8, 4, 3, 7, g=x)
        e = rel(got[x], ref.alpha)
        _say(f"  slice {x}: rel L2 {e:.3e}")
        assert e < 1e-4, (x, e)


def test_readout_ifft_argument_errors():
    import torch
    a = torch.zeros((2, 10, 100), dtype=torch.complex64, device="cuda")
    with pytest.raises(T.T2SError):
        T.t2s_readout_ifft(a, torch.zeros((100, 2, 10), dtype=torch.complex64, device="cuda"))   # length 100
    b = torch.zeros((2, 10, 64), dtype=torch.complex64, device="cuda")
    with pytest.raises(T.T2SError):
        T.t2s_readout_ifft(b, b.view(64, 2, 10))                                               # in place
