"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test targets one oracle function and is chosen so that a plausible mistake
(a dropped term, a wrong sign or index, a transposed operand) fails it.
"""

import os

import numpy as np
import pytest

from oracle import t2s as O

HERE = os.path.dirname(os.path.abspath(__file__))


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def small_problem(rng, ny=16, nz=24, C=3, T=6, K=3, frac=0.3):
    phi, _ = np.linalg.qr(rng.standard_normal((T, K)))
    sens = crandn(rng, C, ny, nz)
    sens /= np.sqrt((np.abs(sens) ** 2).sum(0))[None]
    masks = rng.random((T, ny, nz)) < frac
    return phi, sens, masks


# --- T1: centred DFT against the direct DFT matrix of its definition -------------------


def dft_matrix(n):
    j = np.arange(n)[:, None] - n // 2
    i = np.arange(n)[None, :] - n // 2
    return np.exp(-2j * np.pi * j * i / n) / np.sqrt(n)


@pytest.mark.parametrize("ny,nz", [(4, 4), (6, 10), (12, 8), (12, 20), (24, 40), (10, 6), (26, 30)])
def test_fft2c_matches_direct_dft(ny, nz):
    rng = np.random.default_rng(ny * 100 + nz)
    x = crandn(rng, 2, ny, nz)
    Dy, Dz = dft_matrix(ny), dft_matrix(nz)
    # brute force double sum for one image, matrix form for the other
    X0 = np.zeros((ny, nz), dtype=complex)
    for jy in range(ny):
        for jz in range(nz):
            X0[jy, jz] = np.sum(Dy[jy][:, None] * Dz[jz][None, :] * x[0])
    assert rel(O.fft2c(x)[0], X0) < 1e-12
    assert rel(O.fft2c(x)[1], Dy @ x[1] @ Dz.T) < 1e-12
    assert rel(O.ifft2c(O.fft2c(x)), x) < 1e-12
    assert rel(O.ifft2c(x)[1], Dy.conj().T @ x[1] @ Dz.conj()) < 1e-12


def test_fft2c_paper_grid_matches_direct_dft():
    # the paper's 260 x 240 slice grid (260 = 4 5 13, 240 = 16 15), matrix form
    ny, nz = 240, 260
    rng = np.random.default_rng(260)
    x = crandn(rng, ny, nz)
    Dy, Dz = dft_matrix(ny), dft_matrix(nz)
    assert rel(O.fft2c(x), Dy @ x @ Dz.T) < 1e-12
    jy, jz = 7, 201
    brute = np.sum(Dy[jy][:, None] * Dz[jz][None, :] * x)
    assert abs(O.fft2c(x)[jy, jz] - brute) < 1e-12 * abs(brute)


@pytest.mark.parametrize("nx", [4, 6, 16, 20])
def test_readout_ifft_matches_inverse_dft(nx):
    # decoupling the readout (Sec. II-A end): inverse of the centred unitary DFT,
    # against the conjugate transpose of the direct DFT matrix, a brute-force sum and
    # the forward transform
    rng = np.random.default_rng(nx)
    k = crandn(rng, 2, 5, nx)
    out = O.readout_ifft(k)
    assert out.shape == (nx, 2, 5)
    D = dft_matrix(nx)
    assert rel(out, np.moveaxis(k @ D.conj(), -1, 0)) < 1e-12
    x, c, p = nx // 2 + 1, 1, 3
    brute = sum(k[c, p, j] * np.exp(2j * np.pi * (j - nx // 2) * (x - nx // 2) / nx) for j in range(nx)) / np.sqrt(nx)
    assert abs(out[x, c, p] - brute) < 1e-12 * abs(brute)
    assert rel(np.moveaxis(out, 0, -1) @ D.T, k) < 1e-12


def test_haar_closed_forms_and_orthonormality():
    # a constant image has only an approximation band (2 c per 2 x 2 block for the
    # orthonormal transform); a +-1 pattern along z only the z-detail band
    LL, LH, HL, HH = O.haar2(np.full((4, 6), 3.0 + 1j))
    assert np.allclose(LL, 2 * (3.0 + 1j)) and not LH.any() and not HL.any() and not HH.any()
    z = np.tile([1.0, -1.0, 1.0, -1.0], (4, 1))
    LL, LH, HL, HH = O.haar2(z)
    assert not LL.any() and np.allclose(LH, 2.0) and not HL.any() and not HH.any()
    rng = np.random.default_rng(25)
    x = crandn(rng, 3, 16, 8)
    parts = O.haar2(x)
    assert abs(sum(np.linalg.norm(p) ** 2 for p in parts) - np.linalg.norm(x) ** 2) < 1e-10 * np.linalg.norm(x) ** 2
    assert rel(O.ihaar2(*parts), x) < 1e-14


@pytest.mark.parametrize("levels", [1, 2, 3, 4])
def test_wavelet_denoise_limits(levels):
    rng = np.random.default_rng(26 + levels)
    x = crandn(rng, 2, 32, 48)
    # no threshold: identity; infinite threshold: every aligned 2^J square becomes its mean
    assert rel(O.wavelet_denoise(x, levels, 0.0), x) < 1e-13
    B = 2 ** levels
    means = x.reshape(2, 32 // B, B, 48 // B, B).mean(axis=(2, 4))
    want = np.repeat(np.repeat(means, B, axis=1), B, axis=2)
    assert rel(O.wavelet_denoise(x, levels, 1e30), want) < 1e-13
    # shrinking never increases the energy of the detail bands, so the result is closer
    # to the square means than the input is
    y = O.wavelet_denoise(x, levels, 0.5)
    assert np.linalg.norm(y - want) < np.linalg.norm(x - want)


def test_backproject_recovers_images_in_the_subspace():
    rng = np.random.default_rng(27)
    phi, _ = np.linalg.qr(rng.standard_normal((12, 3)))
    imgs = np.tensordot(phi, crandn(rng, 3, 8, 8), axes=(1, 0))      # a time series in span(Phi)
    alpha = np.tensordot(phi.T, imgs, axes=(1, 0))                    # its coefficients (eq. backproj inverted)
    sel = [1, 5, 11]
    assert rel(O.backproject(alpha, phi[sel]), imgs[sel]) < 1e-13


# --- T2: centring by +-1 modulation (FFTmod, Sec. IV-A) and the shifted kernel -------------


@pytest.mark.parametrize("ny,nz", [(8, 8), (6, 10), (16, 12)])
def test_centring_is_sign_modulation(ny, nz):
    rng = np.random.default_rng(3)
    x = crandn(rng, ny, nz)
    sgn = (-1.0) ** (np.arange(ny)[:, None] + np.arange(nz)[None, :])
    const = (-1.0) ** ((ny + nz) // 2)
    ref = const * sgn * np.fft.fft2(sgn * x) / np.sqrt(ny * nz)
    assert rel(O.fft2c(x), ref) < 1e-12


def test_shifted_kernel_removes_centring():
    # F^H diag(psi) F x == IFFT0( ifftshift(psi) * FFT0(x) ) with plain (uncentred) transforms
    rng = np.random.default_rng(4)
    ny, nz = 12, 16
    x = crandn(rng, ny, nz)
    psi = rng.standard_normal((ny, nz))
    lhs = O.ifft2c(psi * O.fft2c(x))
    rhs = np.fft.ifft2(np.fft.ifftshift(psi) * np.fft.fft2(x))
    assert rel(lhs, rhs) < 1e-12


# --- T3: adjoint identity --------------------------------------------------------------------


def test_adjoint_identity():
    rng = np.random.default_rng(5)
    phi, sens, masks = small_problem(rng)
    K = phi.shape[1]
    a = crandn(rng, K, *sens.shape[1:])
    y = crandn(rng, sens.shape[0], int(masks.sum()))
    lhs = np.vdot(y, O.forward(a, sens, phi, masks))          # <y, A a>
    rhs = np.vdot(O.adjoint(y, sens, phi, masks), a)          # <A^H y, a>
    assert abs(lhs - rhs) / abs(lhs) < 1e-12


def test_forward_samples_in_mask_order():
    # one nonzero coefficient image, one coil of ones, one echo: samples are F(alpha)[mask] row-major
    rng = np.random.default_rng(6)
    ny, nz, T, K = 8, 8, 2, 1
    phi = np.array([[2.0], [-1.0]])
    sens = np.ones((1, ny, nz), dtype=complex)
    masks = np.zeros((T, ny, nz), dtype=bool)
    masks[0, 1, 5] = masks[0, 3, 2] = True
    masks[1, 0, 0] = True
    a = crandn(rng, K, ny, nz)
    Fa = O.fft2c(a[0])
    y = O.forward(a, sens, phi, masks)[0]
    assert np.allclose(y, [2 * Fa[1, 5], 2 * Fa[3, 2], -Fa[0, 0]], rtol=1e-13)


# --- T4: the subspace commutes with coils and Fourier transform (Sec. IV-B) ---------------


def test_commute():
    rng = np.random.default_rng(7)
    phi, sens, _ = small_problem(rng)
    a = crandn(rng, phi.shape[1], *sens.shape[1:])
    for c in range(sens.shape[0]):
        lhs = O.fft2c(sens[c][None] * np.einsum("tk,kyz->tyz", phi, a))
        rhs = np.einsum("tk,kyz->tyz", phi, O.fft2c(sens[c][None] * a))
        assert rel(lhs, rhs) < 1e-12


# --- T5: space-time kernel route of the normal operator -------------------------------------


def test_psi_normal_equals_explicit():
    rng = np.random.default_rng(8)
    phi, sens, masks = small_problem(rng)
    a = crandn(rng, phi.shape[1], *sens.shape[1:])
    psi = O.space_time_kernel(phi, masks)
    assert rel(O.normal_psi(a, sens, psi), O.normal_explicit(a, sens, phi, masks)) < 1e-12


def test_psi_real_symmetric_and_full_sampling():
    rng = np.random.default_rng(9)
    phi, sens, masks = small_problem(rng)
    psi = O.space_time_kernel(phi, masks)
    assert np.isrealobj(psi)
    assert np.array_equal(psi, psi.transpose(1, 0, 2, 3))
    # brute force one location
    n = (3, 5)
    brute = sum(np.outer(phi[t], phi[t]) for t in range(phi.shape[0]) if masks[t][n])
    assert np.allclose(psi[:, :, n[0], n[1]], brute, atol=1e-14)
    full = np.ones_like(masks)
    psi_full = O.space_time_kernel(phi, full)
    eye = np.eye(phi.shape[1])[:, :, None, None]
    assert np.allclose(psi_full, eye, atol=1e-13)         # Phi has orthonormal columns
    a = crandn(rng, phi.shape[1], *sens.shape[1:])
    assert rel(O.normal_psi(a, sens, psi_full), a) < 1e-12   # SoS coils: A^H A = I


# --- T7: LLR prox ------------------------------------------------------------------------------


def test_svt_closed_forms():
    rng = np.random.default_rng(10)
    B, K = 64, 4
    u = crandn(rng, B)
    u /= np.linalg.norm(u)
    v = crandn(rng, K)
    v /= np.linalg.norm(v)
    for sigma, tau in [(3.0, 0.01), (0.5, 0.1), (0.05, 0.1)]:
        X = sigma * np.outer(u, v.conj())
        assert rel(O.svt(X, tau) + 1e-300, max(sigma - tau, 0.0) * np.outer(u, v.conj()) + 1e-300) < 1e-12 \
            or (sigma <= tau and np.abs(O.svt(X, tau)).max() < 1e-14)
    # prescribed singular values through random unitary factors
    U, _ = np.linalg.qr(crandn(rng, B, K))
    V, _ = np.linalg.qr(crandn(rng, K, K))
    s = np.array([2.0, 0.7, 0.15, 0.02])
    X = (U * s) @ V.conj().T
    assert rel(O.svt(X, 0.1), (U * np.maximum(s - 0.1, 0)) @ V.conj().T) < 1e-12
    assert rel(O.svt(X, 0.0), X) < 1e-12
    assert np.abs(O.svt(np.zeros((B, K)), 0.1)).max() == 0.0
    # homogeneity and row permutation equivariance
    assert rel(O.svt(3.0 * X, 0.3), 3.0 * O.svt(X, 0.1)) < 1e-12
    perm = rng.permutation(B)
    assert rel(O.svt(X[perm], 0.1), O.svt(X, 0.1)[perm]) < 1e-12


def test_svt_is_the_proximal_map():
    # SVT minimises 1/2||X - Y||^2 + tau ||X||_*; random perturbations never do better
    rng = np.random.default_rng(11)
    Y = crandn(rng, 16, 3)
    tau = 0.8

    def f(X):
        return 0.5 * np.linalg.norm(X - Y) ** 2 + tau * np.linalg.svd(X, compute_uv=False).sum()

    X = O.svt(Y, tau)
    f0 = f(X)
    for scale in (1e-1, 1e-3):
        for _ in range(50):
            assert f(X + scale * crandn(rng, 16, 3)) >= f0 - 1e-12


def test_llr_identity_zero_and_single_vs_explicit():
    rng = np.random.default_rng(12)
    K, ny, nz, b = 3, 16, 24, 8
    v = crandn(rng, K, ny, nz)
    assert rel(O.llr_prox(v, 0.0, (3, 5), b), v) < 1e-12
    assert np.abs(O.llr_prox(np.zeros_like(v), 0.1, (3, 5), b)).max() == 0.0
    for shift in [(0, 0), (3, 5), (7, 1)]:
        assert rel(O.llr_prox(v, 0.7, shift, b), O.llr_prox_explicit(v, 0.7, shift, b)) < 1e-12


def test_llr_block_membership_under_shift():
    # a rank-1 pattern confined to one shifted block is shrunk by exactly tau there and
    # nothing else moves: pins the block membership rule (rows p*b + i + s_y mod Ny)
    rng = np.random.default_rng(13)
    K, ny, nz, b = 2, 16, 16, 4
    sy, sz = 3, 2
    v = np.zeros((K, ny, nz), dtype=complex)
    rows = (1 * b + np.arange(b) + sy) % ny
    cols = (3 * b + np.arange(b) + sz) % nz        # wraps around
    uvec = crandn(rng, b * b)
    uvec /= np.linalg.norm(uvec)
    wvec = crandn(rng, K)
    wvec /= np.linalg.norm(wvec)
    blk = 2.0 * np.outer(uvec, wvec.conj())        # [B, K], sigma = 2
    v[:, rows[:, None], cols[None, :]] = blk.T.reshape(K, b, b)
    out = O.llr_prox(v, 0.5, (sy, sz), b)
    assert rel(out, 0.75 * v) < 1e-12
    # with a different shift the pattern straddles blocks: no longer a pure rescale
    out2 = O.llr_prox(v, 0.5, (0, 0), b)
    assert rel(out2, 0.75 * v) > 1e-3


def test_llr_value_matches_svd():
    rng = np.random.default_rng(14)
    v = crandn(rng, 2, 8, 8)
    val = O.llr_value(v, (1, 2), 4)
    brute = 0.0
    w = np.roll(v, (-1, -2), axis=(1, 2))
    for p in range(2):
        for q in range(2):
            X = w[:, 4 * p:4 * p + 4, 4 * q:4 * q + 4].reshape(2, 16).T
            brute += np.linalg.svd(X, compute_uv=False).sum()
    assert abs(val - brute) < 1e-12 * brute


# --- T9: CG ---------------------------------------------------------------------------------


def test_cg_solves_hpd_system():
    rng = np.random.default_rng(15)
    n = 12
    Q = crandn(rng, n, n)
    M = Q @ Q.conj().T + 0.5 * np.eye(n)
    b = crandn(rng, n)
    x = O.cg(lambda v: M @ v, np.zeros(n, dtype=complex), b, 3 * n)
    assert rel(x, np.linalg.solve(M, b)) < 1e-10
    # a few iterations reduce the M-norm error monotonically
    xs = [O.cg(lambda v: M @ v, np.zeros(n, dtype=complex), b, k) for k in range(1, 6)]
    xt = np.linalg.solve(M, b)
    errs = [np.vdot(x - xt, M @ (x - xt)).real for x in xs]
    assert all(e1 <= e0 * (1 + 1e-12) for e0, e1 in zip(errs, errs[1:]))


def test_cg_one_step_exact_for_scaled_identity():
    rng = np.random.default_rng(16)
    phi, sens, _ = small_problem(rng)
    full = np.ones((phi.shape[0],) + sens.shape[1:], dtype=bool)
    psi = O.space_time_kernel(phi, full)
    rho = 0.1
    b = crandn(rng, phi.shape[1], *sens.shape[1:])
    x = O.cg(lambda v: O.normal_psi(v, sens, psi) + rho * v, np.zeros_like(b), b, 1)
    assert rel(x, b / (1 + rho)) < 1e-12


# --- T12: shift schedule -------------------------------------------------------------------


def test_splitmix64_golden():
    vals = [int(l) for l in open(os.path.join(HERE, "golden", "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    state, M = 1234567, (1 << 64) - 1
    for v in vals:
        assert O.splitmix64(state) == v
        state = (state + 0x9E3779B97F4A7C15) & M


def test_block_shift_range_and_spread():
    seen = set()
    for k in range(400):
        sy, sz = O.block_shift(0, 3, k, 8)
        assert 0 <= sy < 8 and 0 <= sz < 8
        seen.add((sy, sz))
    assert len(seen) > 50
    assert O.block_shift(1, 0, 0, 8) != O.block_shift(1, 1, 0, 8) or O.block_shift(1, 0, 1, 8) != O.block_shift(1, 1, 1, 8)


# --- T10 / T11: ADMM ------------------------------------------------------------------------


def test_admm_exact_recovery_full_sampling():
    rng = np.random.default_rng(17)
    phi, sens, _ = small_problem(rng, ny=16, nz=16)
    full = np.ones((phi.shape[0], 16, 16), dtype=bool)
    a_true = crandn(rng, phi.shape[1], 16, 16)
    y = O.forward(a_true, sens, phi, full)
    res = O.admm(y, sens, phi, full, lam=0.0, rho=0.1, b=8, n_outer=12, n_cg=5, seed=0)
    assert rel(res.alpha, a_true) < 1e-10


def _explicit_matrix(sens, phi, masks):
    K = phi.shape[1]
    ny, nz = sens.shape[1:]
    cols = []
    for i in range(K * ny * nz):
        e = np.zeros(K * ny * nz, dtype=complex)
        e[i] = 1.0
        cols.append(O.forward(e.reshape(K, ny, nz), sens, phi, masks).reshape(-1))
    return np.stack(cols, axis=1)


def test_admm_lambda0_is_min_norm_least_squares():
    rng = np.random.default_rng(18)
    phi, sens, masks = small_problem(rng, ny=8, nz=8, C=2, T=4, K=2, frac=0.5)
    A = _explicit_matrix(sens, phi, masks)
    y = crandn(rng, 2, int(masks.sum()))
    x_ls = np.linalg.lstsq(A, y.reshape(-1), rcond=None)[0]
    res = O.admm(y, sens, phi, masks, lam=0.0, rho=0.1, b=4, n_outer=400, n_cg=20, seed=0)
    assert rel(res.alpha.reshape(-1), x_ls) < 1e-8


@pytest.mark.slow
def test_admm_matches_fista_objective_at_fixed_shift():
    rng = np.random.default_rng(19)
    phi, sens, masks = small_problem(rng, ny=8, nz=8, C=2, T=4, K=2, frac=0.35)
    a_true = crandn(rng, 2, 8, 8)
    y = O.forward(a_true, sens, phi, masks) + 0.05 * crandn(rng, 2, int(masks.sum()))
    lam, shift = 0.3, (1, 3)
    r_admm = O.admm(y, sens, phi, masks, lam=lam, rho=0.5, b=4, n_outer=3000, n_cg=20, seed=0,
                    fixed_shift=shift)
    x_f = O.fista(y, sens, phi, masks, lam=lam, b=4, n_iter=6000, shift=shift)
    fa = O.objective(r_admm.alpha, y, sens, phi, masks, lam, shift, 4)
    ff = O.objective(x_f, y, sens, phi, masks, lam, shift, 4)
    assert abs(fa - ff) / abs(ff) < 1e-8


# --- FISTA (the paper's solver, Sec. II-A) and its step size --------------------------------


def test_lipschitz_closed_form_full_sampling():
    # full sampling and an orthonormal basis make Psi = I, so A^H A multiplies every
    # pixel by sum_c |S_c|^2: its largest eigenvalue is the largest such sum
    rng = np.random.default_rng(23)
    phi, _, _ = small_problem(rng, ny=16, nz=16)
    sens = crandn(rng, 3, 16, 16)
    sens[:, 5, 7] *= 3.0                      # one pixel well above the rest
    full = np.ones((phi.shape[0], 16, 16), dtype=bool)
    psi = O.space_time_kernel(phi, full)
    L = O.lipschitz(sens, psi, crandn(rng, phi.shape[1], 16, 16), 60)
    assert abs(L - (np.abs(sens) ** 2).sum(0).max()) < 1e-10 * L
    # zero start vector: no direction to iterate on
    assert O.lipschitz(sens, psi, np.zeros((phi.shape[1], 16, 16), complex), 3) == 0.0


def test_lipschitz_matches_largest_eigenvalue():
    rng = np.random.default_rng(22)
    phi, sens, masks = small_problem(rng, ny=8, nz=8, C=2, T=4, K=2, frac=0.5)
    A = _explicit_matrix(sens, phi, masks)
    lmax = np.linalg.eigvalsh(A.conj().T @ A)[-1]
    L = O.lipschitz(sens, O.space_time_kernel(phi, masks), crandn(rng, 2, 8, 8), 4000)
    assert L <= lmax * (1 + 1e-12) and abs(L - lmax) < 1e-5 * lmax


def test_fista_shift_schedule_lambda0_is_min_norm_least_squares():
    # without the regulariser the shifts do nothing and FISTA from 0 converges to the
    # minimum-norm least-squares solution of the explicit system
    rng = np.random.default_rng(22)
    phi, sens, masks = small_problem(rng, ny=8, nz=8, C=2, T=4, K=2, frac=0.5)
    A = _explicit_matrix(sens, phi, masks)
    y = crandn(rng, 2, int(masks.sum()))
    x_ls = np.linalg.lstsq(A, y.reshape(-1), rcond=None)[0]
    step = 1.0 / np.linalg.eigvalsh(A.conj().T @ A)[-1]
    x = O.fista(y, sens, phi, masks, lam=0.0, b=4, n_iter=2000, seed=3, g=1, step=step)
    assert rel(x.reshape(-1), x_ls) < 1e-10


def test_fista_first_step_is_a_prox_gradient_step_at_the_scheduled_shift():
    # y_0 = x_0 and t_0 = 1 give zero momentum in the first step, so one iteration is
    # one proximal-gradient step at shift block_shift(seed, g, 0); it differs from the
    # same step at another shift whenever the threshold bites
    rng = np.random.default_rng(24)
    phi, sens, masks = small_problem(rng, ny=16, nz=16, C=2, T=4, K=2, frac=0.4)
    y = O.forward(crandn(rng, 2, 16, 16), sens, phi, masks)
    x0 = crandn(rng, 2, 16, 16)
    seed, g, lam, step = 5, 7, 0.5, 0.9
    x1 = O.fista(y, sens, phi, masks, lam=lam, b=8, n_iter=1, seed=seed, g=g, step=step, alpha0=x0)
    grad = O.normal_explicit(x0, sens, phi, masks) - O.adjoint(y, sens, phi, masks)
    sh = O.block_shift(seed, g, 0, 8)
    assert rel(x1, O.llr_prox_explicit(x0 - step * grad, lam * step, sh, 8)) < 1e-12
    other = ((sh[0] + 1) % 8, sh[1])
    assert rel(x1, O.llr_prox_explicit(x0 - step * grad, lam * step, other, 8)) > 1e-3


def test_admm_tolerance_mode_rules():
    # freeze happens only at check points; under random shifts the residual stalls
    # above tol, so the run freezes first and then stops once converged
    rng = np.random.default_rng(20)
    phi, sens, masks = small_problem(rng, ny=16, nz=16, C=2, T=4, K=2, frac=0.4)
    a_true = crandn(rng, 2, 16, 16)
    y = O.forward(a_true, sens, phi, masks)
    res = O.admm(y, sens, phi, masks, lam=0.01, rho=0.1, b=8, n_outer=300, n_cg=5, seed=4,
                 tol=1e-4, check_every=5)
    assert res.k_freeze >= 0 and (res.k_freeze + 1) % 5 == 0
    assert res.n_outer % 5 == 0 and res.n_outer < 300
    assert res.history[-1]["res"] <= 1e-4
    shifts_after = {h["shift"] for h in res.history[res.k_freeze:]}
    assert len(shifts_after) == 1


def test_admm_tolerance_degenerate_slices():
    rng = np.random.default_rng(21)
    phi, sens, masks = small_problem(rng, ny=16, nz=16, C=2, T=4, K=2, frac=0.4)
    P = int(masks.sum())
    # no signal: alpha = z = u = 0 exactly, residuals 0, stop at the first check
    res = O.admm(np.zeros((2, P), np.complex128), sens, phi, masks, lam=0.01, rho=0.1, b=8, n_outer=300, n_cg=5,
                 seed=4, tol=1e-4, check_every=5)
    assert res.n_outer == 5 and not np.any(res.alpha) and res.history[-1]["res"] == 0.0
    # every block far below the threshold: the solution is zero; the scale floor
    # (a fraction of ||A^H y||) lets the relative residual reach tol before the cap
    y = O.forward(1e-3 * crandn(rng, 2, 16, 16), sens, phi, masks)
    res = O.admm(y, sens, phi, masks, lam=10.0, rho=0.1, b=8, n_outer=300, n_cg=5, seed=4, tol=1e-4,
                 check_every=5)
    assert res.n_outer < 300 and res.history[-1]["res"] <= 1e-4
    assert np.linalg.norm(res.z) == 0.0
    assert np.linalg.norm(res.alpha) <= 1e-4 * 0.01 * np.linalg.norm(O.adjoint(y, sens, phi, masks)) * 1.0001


# --- partial LLR blocks (a block edge that does not divide the grid) --------------------


@pytest.mark.parametrize("n,b,sh", [(20, 8, 3), (260, 12, 11), (240, 12, 0), (16, 16, 5), (9, 4, 2)])
def test_block_ranges_partition_the_axis(n, b, sh):
    ranges = O.block_ranges(n, b, sh)
    allidx = np.concatenate(ranges)
    assert sorted(allidx.tolist()) == list(range(n))          # every index in exactly one block
    sizes = [r.size for r in ranges]
    assert sizes[:-1] == [b] * (len(ranges) - 1) and sizes[-1] == n - (len(ranges) - 1) * b
    assert ranges[0][0] == sh % n                              # block 0 starts at the shift


def test_llr_partial_blocks_single_pass_equals_explicit():
    # modular gather of the single pass vs circular shift + contiguous tiles cut short
    rng = np.random.default_rng(21)
    v = crandn(rng, 3, 20, 28)
    for shift in ((0, 0), (3, 5), (7, 7)):
        assert rel(O.llr_prox(v, 0.8, shift, 8), O.llr_prox_explicit(v, 0.8, shift, 8)) < 1e-12
    v = crandn(rng, 4, 24, 26)
    assert rel(O.llr_prox(v, 0.5, (11, 4), 12), O.llr_prox_explicit(v, 0.5, (11, 4), 12)) < 1e-12


def test_llr_partial_block_rank_one_shrunk_by_tau():
    # a rank-1 pattern sigma u v^H filling exactly the partial corner block (wrapped by
    # the shift) and zero elsewhere comes back as (sigma - tau) u v^H; other blocks stay 0
    K, Ny, Nz, b, shift = 3, 20, 26, 8, (6, 5)
    rows = O.block_ranges(Ny, b, shift[0])[-1]
    cols = O.block_ranges(Nz, b, shift[1])[-1]
    assert rows.size == 4 and cols.size == 2
    rng = np.random.default_rng(22)
    uvec = crandn(rng, rows.size * cols.size)
    uvec /= np.linalg.norm(uvec)
    vvec = crandn(rng, K)
    vvec /= np.linalg.norm(vvec)
    sigma, tau = 3.0, 0.7
    X = sigma * np.outer(uvec, vvec.conj())                  # [voxels, K]
    v = np.zeros((K, Ny, Nz), dtype=complex)
    v[:, rows[:, None], cols[None, :]] = X.T.reshape(K, rows.size, cols.size)
    out = O.llr_prox(v, tau, shift, b)
    assert rel(out, v * (sigma - tau) / sigma) < 1e-12


# --- soft-SENSE: M = 2 coil-map sets (Sec. II-A) -------------------------------------------


def test_two_map_sets_adjoint_identity_and_routes():
    rng = np.random.default_rng(31)
    phi, s1, masks = small_problem(rng, ny=12, nz=14, C=3, T=6, K=3)
    sens = np.stack([s1, 0.5 * crandn(rng, *s1.shape)], axis=1)          # [C, 2, Ny, Nz]
    alpha = crandn(rng, 2, 3, 12, 14)
    y = crandn(rng, 3, int(masks.sum()))
    lhs = np.vdot(y, O.forward(alpha, sens, phi, masks))
    rhs = np.vdot(O.adjoint(y, sens, phi, masks), alpha)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    psi = O.space_time_kernel(phi, masks)
    assert rel(O.normal_psi(alpha, sens, psi), O.normal_explicit(alpha, sens, phi, masks)) < 1e-12


def test_two_map_sets_reduce_to_one():
    # a second map set of zeros leaves the first set's problem unchanged and gets nothing
    # back; coil images are the sum over map sets (swapping the sets swaps the results)
    rng = np.random.default_rng(32)
    phi, s1, masks = small_problem(rng, ny=12, nz=10, C=2, T=5, K=2)
    alpha = crandn(rng, 2, 2, 12, 10)
    psi = O.space_time_kernel(phi, masks)
    sens = np.stack([s1, np.zeros_like(s1)], axis=1)
    out = O.normal_psi(alpha, sens, psi)
    assert rel(out[0], O.normal_psi(alpha[0], s1, psi)) < 1e-12
    assert np.abs(out[1]).max() == 0
    y = O.forward(alpha, sens, phi, masks)
    assert rel(y, O.forward(alpha[0], s1, phi, masks)) < 1e-12
    s2 = crandn(rng, *s1.shape)
    both = np.stack([s1, s2], axis=1)
    swapped = np.stack([s2, s1], axis=1)
    assert rel(O.forward(alpha, both, phi, masks), O.forward(alpha[::-1], swapped, phi, masks)) < 1e-12
    a = O.adjoint(y, both, phi, masks)
    assert rel(a[0], O.adjoint(y, s1, phi, masks)) < 1e-12 and rel(a[1], O.adjoint(y, s2, phi, masks)) < 1e-12


def test_two_map_sets_llr_per_set():
    rng = np.random.default_rng(33)
    v = crandn(rng, 2, 3, 16, 24)
    out = O.llr_prox(v, 0.6, (3, 5), 8)
    assert rel(out[0], O.llr_prox(v[0], 0.6, (3, 5), 8)) < 1e-14
    assert rel(out[1], O.llr_prox(v[1], 0.6, (3, 5), 8)) < 1e-14


def test_admm_residuals_closed_forms():
    # r_p = ||alpha - z|| / d, r_d = ||z - z_prev|| / d, d = max(||alpha||, ||z||, floor ||b0||)
    rng = np.random.default_rng(40)
    z = crandn(rng, 3, 8, 8)
    nz = np.linalg.norm(z)
    rp, rd = O.admm_residuals(z, z, z, 0 * z, 0.1)
    assert rp == 0.0 and rd == 0.0
    # alpha = 2 z: d = ||alpha|| = 2 ||z||, r_p = 1/2; z_prev = 0: r_d = ||z|| / (2 ||z||)
    rp, rd = O.admm_residuals(2 * z, z, 0 * z, 0 * z, 0.1)
    assert abs(rp - 0.5) < 1e-14 and abs(rd - 0.5) < 1e-14
    # the scale is the larger of the two norms, whichever it is
    rp, _ = O.admm_residuals(0.5 * z, z, z, 0 * z, 0.1)
    assert abs(rp - 0.5 * nz / nz) < 1e-14
    # a tiny solution: the floor O.RESIDUAL_SCALE_FLOOR ||b0|| takes over as the scale
    rp, rd = O.admm_residuals(1e-6 * z, 0 * z, 0 * z, 0 * z, 0.1, b0_norm=nz)
    assert abs(rp - 1e-6 / O.RESIDUAL_SCALE_FLOOR) < 1e-12 and rd == 0.0
    # all zero, no signal: both residuals 0 (the empty slice stops at its first check)
    assert O.admm_residuals(0 * z, 0 * z, 0 * z, 0 * z, 0.1) == (0.0, 0.0)
