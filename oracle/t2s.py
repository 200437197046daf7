"""FP64 oracle of the T2-Shuffling per-slice reconstruction (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and ``bench.py``'s ``cpu_baseline`` leg, never by the product path.

Everything here is plain NumPy in complex128 / float64, written to be read
against the paper (Anderson, Tamir et al., "T2 Shuffling ... distributed
reconstruction", arXiv 1809.04195):

* forward model of one readout slice, Sec. II-A eq. (coilmodel) with the
  temporal subspace of Sec. II-B eq. (backproj): y = P F S Phi alpha;
* problem solved, Sec. II-B eq. (t2shpics): 1/2 ||y - P F S Phi alpha||^2
  + lambda * sum_blocks ||R(alpha)||_* ;
* space-time kernel Psi(n) = Phi^T P(n) Phi of Sec. IV-B (real, symmetric);
* non-overlapping LLR blocks under a random circular shift each iteration,
  Sec. II-B (end) and the single-pass variant of Sec. IV-C;
* ADMM (scaled form) with a CG inner solve on A^H A + rho I.  The paper itself
  runs FISTA (Sec. II-A); ``fista`` is provided for cross-checking objectives.

Array conventions (shared with the C ABI, as plain data):
  alpha        complex [K, Ny, Nz]          subspace coefficient images
  sens         complex [C, Ny, Nz]          coil maps S_c (M = 1 map set), or
               complex [C, M, Ny, Nz]       M soft-SENSE map sets (alpha then [M, K, Ny, Nz])
  phi          real    [T, K]               temporal basis
  masks        bool    [T, Ny, Nz]          centred sampling masks, DC at (Ny/2, Nz/2)
  samples      complex [C, P_tot]           measured k-space in *mask order*:
                                            echo-major, then row-major (y, z)
                                            position inside mask_t.
Frequency index j of a mask / k-space array means frequency j - N/2 (centred).
"""

from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------------------
# Centred unitary 2D DFT  (Sec. II-A: F is the 2D DFT; the pipeline uses unitary
# transforms on centred data, Sec. III-B and the FFTmod step of Sec. IV-A)
# ---------------------------------------------------------------------------


def fft2c(x: np.ndarray) -> np.ndarray:
    """Centred orthonormal 2D DFT over the last two axes.

    (F x)[j] = N^{-1/2} sum_i x[i] exp(-2 pi i (j - N/2)(i - N/2) / N) per axis,
    which for even N equals fftshift(fft2(ifftshift(x))) / sqrt(N).
    """
    ax = (-2, -1)
    return np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(x, axes=ax), axes=ax, norm="ortho"), axes=ax)


def ifft2c(X: np.ndarray) -> np.ndarray:
    """Adjoint (= inverse) of ``fft2c``."""
    ax = (-2, -1)
    return np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(X, axes=ax), axes=ax, norm="ortho"), axes=ax)


# ---------------------------------------------------------------------------
# Sampling pattern in truncated form (Sec. II-A: P in {0,1}^{P x N})
# ---------------------------------------------------------------------------


def mask_order(masks: np.ndarray):
    """Return (echo index, flat location) of every sample, in mask order.

    Mask order is echo-major, then row-major (y, z) location inside mask_t.
    """
    masks = np.asarray(masks).astype(bool)
    T = masks.shape[0]
    t_idx, loc = [], []
    for t in range(T):
        flat = np.flatnonzero(masks[t].reshape(-1))
        t_idx.append(np.full(flat.size, t, dtype=np.int64))
        loc.append(flat)
    return np.concatenate(t_idx), np.concatenate(loc)


# ---------------------------------------------------------------------------
# Forward and adjoint operators  (eq. coilmodel + eq. backproj, i.e. A = P F S Phi)
# ---------------------------------------------------------------------------


# Soft-SENSE (Sec. II-A): with M sets of coil maps, sens is [C, M, Ny, Nz] and the
# unknown has one set of K coefficient images per map set, alpha [M, K, Ny, Nz]; coil c
# sees sum_m S_(c,m) x_m.  A [C, Ny, Nz] sens (M = 1) goes with alpha [K, Ny, Nz].


def _maps(alpha, sens):
    """(alpha [M, K, Ny, Nz], sens [C, M, Ny, Nz], single-set flag) in complex128."""
    alpha = np.asarray(alpha, dtype=np.complex128)
    sens = np.asarray(sens, dtype=np.complex128)
    if sens.ndim == 3:
        return alpha[None], sens[:, None], True
    return alpha, sens, False


def forward(alpha, sens, phi, masks):
    """A alpha: samples[c, p] = (F(sum_m S_cm x_mt))[loc_p] with x_mt = sum_k Phi[t,k] alpha_mk, t = t_p."""
    alpha, sens, _ = _maps(alpha, sens)
    phi = np.asarray(phi, dtype=np.float64)
    T = phi.shape[0]
    C, M, Ny, Nz = sens.shape
    t_of, loc = mask_order(masks)
    x = np.einsum("tk,mkyz->mtyz", phi, alpha)                  # back-projection to echoes, per map set
    out = np.empty((C, t_of.size), dtype=np.complex128)
    for c in range(C):
        img = np.einsum("myz,mtyz->tyz", sens[c], x)           # coil image sum_m S_cm x_m
        kspace = fft2c(img).reshape(T, Ny * Nz)                 # [T, N] full k-space
        out[c] = kspace[t_of, loc]                              # P: keep sampled entries
    return out


def adjoint(samples, sens, phi, masks):
    """A^H y: zero-fill each echo, project onto the basis, inverse DFT, combine each map
    set's coils."""
    samples = np.asarray(samples, dtype=np.complex128)
    _, sens4, single = _maps(np.zeros(1), sens)
    phi = np.asarray(phi, dtype=np.float64)
    T, K = phi.shape
    C, M, Ny, Nz = sens4.shape
    t_of, loc = mask_order(masks)
    alpha = np.zeros((M, K, Ny, Nz), dtype=np.complex128)
    for c in range(C):
        full = np.zeros((T, Ny * Nz), dtype=np.complex128)
        full[t_of, loc] = samples[c]                            # P^H: zero-fill
        proj = np.einsum("tk,tn->kn", phi, full).reshape(K, Ny, Nz)   # Phi^T
        img = ifft2c(proj)                                      # F^H
        for m in range(M):
            alpha[m] += np.conj(sens4[c, m])[None] * img        # S_cm^H
    return alpha[0] if single else alpha


# ---------------------------------------------------------------------------
# Space-time kernel and the normal operator (Sec. IV-B, eqs. commute / normaleq)
# ---------------------------------------------------------------------------


def space_time_kernel(phi, masks):
    """Psi(n) = Phi^T P(n) Phi = sum_{t : m_t(n)=1} phi_t^T phi_t, shape [K, K, Ny, Nz] (real)."""
    phi = np.asarray(phi, dtype=np.float64)
    m = np.asarray(masks).astype(np.float64)
    return np.einsum("tk,tl,tyz->klyz", phi, phi, m)


def normal_explicit(alpha, sens, phi, masks):
    """Route (i): A^H (A alpha)."""
    return adjoint(forward(alpha, sens, phi, masks), sens, phi, masks)


def normal_psi(alpha, sens, psi):
    """Route (ii): N(alpha)_mk = sum_c conj(S_cm) F^H( sum_l Psi_kl F(sum_m' S_cm' alpha_m'l) )."""
    alpha, sens, single = _maps(alpha, sens)
    out = np.zeros_like(alpha)
    for c in range(sens.shape[0]):
        ks = fft2c(np.einsum("myz,mkyz->kyz", sens[c], alpha))  # [K, Ny, Nz]
        mixed = ifft2c(np.einsum("klyz,lyz->kyz", psi, ks))
        for m in range(sens.shape[1]):
            out[m] += np.conj(sens[c, m])[None] * mixed
    return out[0] if single else out


# ---------------------------------------------------------------------------
# Locally-low-rank proximal map  (eq. llr; random shift + non-overlapping b x b
# blocks, Sec. II-B; single pass over the images, Sec. IV-C)
# ---------------------------------------------------------------------------


def svt(X: np.ndarray, tau: float) -> np.ndarray:
    """Singular-value soft threshold of a matrix: U diag(max(s - tau, 0)) V^H."""
    U, s, Vh = np.linalg.svd(X, full_matrices=False)
    return (U * np.maximum(s - tau, 0.0)) @ Vh


def block_ranges(n, b, s):
    """Index sets of the blocks along one axis of length n: block p holds
    (p*b + i + s) mod n for the i in [0, b) with p*b + i < n.  When b does not divide n
    the last block is partial (n - (ceil(n/b) - 1) b entries); the paper's 260-point
    axis with 12-point blocks has 21 full blocks and one of 8 (the paper does not say
    how it treats the remainder)."""
    return [(p * b + np.arange(min(b, n - p * b)) + s) % n for p in range((n + b - 1) // b)]


def llr_prox(v, tau, shift, b):
    """Single-pass LLR prox: gather each shifted block, threshold, scatter back.

    Block (p, q) holds rows (p*b + i + s_y) mod Ny and columns (q*b + j + s_z) mod Nz,
    i, j in [0, b) (partial blocks at the end of an axis b does not divide, see
    ``block_ranges``); its matrix has one row per voxel (row-major inside the block)
    and one column per coefficient image.
    """
    v = np.asarray(v, dtype=np.complex128)
    if v.ndim == 4:   # one prox per map set (soft-SENSE): the blocks of each set's K images
        return np.stack([llr_prox(vm, tau, shift, b) for vm in v])
    K, Ny, Nz = v.shape
    sy, sz = shift
    out = np.empty_like(v)
    for rows in block_ranges(Ny, b, sy):
        for cols in block_ranges(Nz, b, sz):
            blk = v[:, rows[:, None], cols[None, :]]           # [K, by, bz]
            X = blk.reshape(K, -1).T                            # [by bz, K]
            out[:, rows[:, None], cols[None, :]] = svt(X, tau).T.reshape(blk.shape)
    return out


def llr_prox_explicit(v, tau, shift, b):
    """The same prox written as: circular shift, cut the shifted images into
    contiguous b x b tiles (the tiles of the last row / column cut short where b does
    not divide the grid), threshold each, shift back (the multi-pass form the paper
    replaced)."""
    v = np.asarray(v, dtype=np.complex128)
    K, Ny, Nz = v.shape
    sy, sz = shift
    w = np.roll(v, (-sy, -sz), axis=(1, 2))                     # w[i] = v[i + s]
    res = np.empty_like(w)
    for y0 in range(0, Ny, b):
        for z0 in range(0, Nz, b):
            tile = w[:, y0:y0 + b, z0:z0 + b]
            X = tile.transpose(1, 2, 0).reshape(-1, K)           # voxels row-major, one column per image
            res[:, y0:y0 + b, z0:z0 + b] = svt(X, tau).reshape(tile.shape[1], tile.shape[2], K).transpose(2, 0, 1)
    return np.roll(res, (sy, sz), axis=(1, 2))


def llr_value(alpha, shift, b):
    """sum over the shifted non-overlapping blocks of the nuclear norm (eq. llr, blocked form)."""
    alpha = np.asarray(alpha, dtype=np.complex128)
    if alpha.ndim == 4:
        return sum(llr_value(am, shift, b) for am in alpha)
    K, Ny, Nz = alpha.shape
    sy, sz = shift
    total = 0.0
    for rows in block_ranges(Ny, b, sy):
        for cols in block_ranges(Nz, b, sz):
            X = alpha[:, rows[:, None], cols[None, :]].reshape(K, -1).T
            total += np.linalg.svd(X, compute_uv=False).sum()
    return total


def objective(alpha, samples, sens, phi, masks, lam, shift, b):
    """Value of eq. (t2shpics) with the blocked regulariser at a fixed shift."""
    res = samples - forward(alpha, sens, phi, masks)
    return 0.5 * np.vdot(res, res).real + lam * llr_value(alpha, shift, b)


# ---------------------------------------------------------------------------
# Random block shift: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), counter based
# ---------------------------------------------------------------------------

_M64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """One SplitMix64 output for state x (state advanced by the golden gamma first)."""
    z = (x + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def block_shift(seed: int, g: int, k: int, b: int):
    """Shift (s_y, s_z) in [0, b)^2 of global slice g at outer iteration k.

    h = sm(sm(sm(seed) xor g) xor k); s_y = (h mod 2^32) mod b; s_z = (h >> 32) mod b.
    """
    h = splitmix64(splitmix64(splitmix64(seed & _M64) ^ (g & _M64)) ^ (k & _M64))
    return (h & 0xFFFFFFFF) % b, (h >> 32) % b


# ---------------------------------------------------------------------------
# Conjugate gradient on M = A^H A + rho I
# ---------------------------------------------------------------------------


def cg(apply_m, x0, rhs, n_iter):
    """Plain CG (no preconditioner), warm-started at x0, explicit initial residual.

    <u, v> = sum conj(u) v; the step uses Re<p, Mp>.  Stops early if gamma == 0.
    """
    x = np.array(x0, dtype=np.complex128, copy=True)
    r = rhs - apply_m(x)
    p = r.copy()
    gamma = np.vdot(r, r).real
    for _ in range(n_iter):
        if gamma == 0.0:
            break
        w = apply_m(p)
        pw = np.vdot(p, w).real
        if pw == 0.0:
            break
        a = gamma / pw
        x += a * p
        r -= a * w
        gamma_new = np.vdot(r, r).real
        p = r + (gamma_new / gamma) * p
        gamma = gamma_new
    return x


# ---------------------------------------------------------------------------
# ADMM (scaled form; Boyd et al. 2011, Sec. 3.1.1) for eq. (t2shpics)
# ---------------------------------------------------------------------------


class AdmmResult:
    def __init__(self, alpha, z, u, history, k_freeze, n_outer):
        self.alpha = alpha
        self.z = z
        self.u = u
        self.history = history          # list of dicts, one per outer iteration
        self.k_freeze = k_freeze        # outer index whose shift was frozen (-1: never)
        self.n_outer = n_outer          # outer iterations run


# Floor of the residual scale, as a fraction of ||b0|| = ||A^H y||: a slice whose
# solution is zero (every block below the threshold) would otherwise divide by a
# vanishing ||alpha||.
RESIDUAL_SCALE_FLOOR = 0.01


def admm_residuals(alpha, z, z_prev, u, rho, b0_norm=0.0):
    """Primal residual alpha - z and dual residual rho (z - z_prev) (Boyd et al.,
    Sec. 3.3), both relative to the scale of the solution:
    r_p = ||alpha - z|| / d,  r_d = rho ||z - z_prev|| / (rho d),
    d = max(||alpha||, ||z||, RESIDUAL_SCALE_FLOOR ||b0||)   (0 when d = 0)"""
    na, nz = np.linalg.norm(alpha), np.linalg.norm(z)
    den = max(na, nz, RESIDUAL_SCALE_FLOOR * b0_norm)
    rp = np.linalg.norm(alpha - z) / den if den > 0 else 0.0
    rd = np.linalg.norm(z - z_prev) / den if den > 0 else 0.0
    return rp, rd


def admm(samples, sens, phi, masks, lam, rho, b, n_outer, n_cg, seed, g=0,
         alpha0=None, tol=0.0, freeze_window=5, freeze_stall=0.05, check_every=5,
         fixed_shift=None, replay=None, normal="psi"):
    """Solve eq. (t2shpics) for one slice.

    Per outer iteration k:
      1. alpha <- CG(alpha, b0 + rho (z - u), n_cg) on M = A^H A + rho I
      2. z <- LLR prox with threshold lam/rho at shift(seed, g, k) (or the frozen shift)
      3. u <- u + alpha - z
    Fixed mode (tol == 0): exactly n_outer iterations, a new shift every iteration.
    Tolerance mode (tol > 0): decisions are taken after outer iterations k with
    (k + 1) % check_every == 0, in this order: stop if max(r_p, r_d) <= tol; else,
    if the shift is not frozen yet, freeze it at shift k if max(r_p, r_d) at k
    exceeds (1 - freeze_stall) times its value at k - freeze_window.  n_outer is the
    cap.  (Under random shifts the residual stalls well above tol, so the stop
    normally comes after the freeze; a slice whose residual is exactly zero, such as
    one with no signal, stops at the first check.)
    ``replay`` = (k_freeze, n_run) imposes another run's decisions instead.
    """
    sens = np.asarray(sens, dtype=np.complex128)
    phi = np.asarray(phi, dtype=np.float64)
    K = phi.shape[1]
    Ny, Nz = sens.shape[-2:]
    shape = (K, Ny, Nz) if sens.ndim == 3 else (sens.shape[1], K, Ny, Nz)
    tau = lam / rho
    b0 = adjoint(samples, sens, phi, masks)
    b0_norm = np.linalg.norm(b0)
    if normal == "psi":
        psi = space_time_kernel(phi, masks)

        def apply_m(v):
            return normal_psi(v, sens, psi) + rho * v
    else:
        def apply_m(v):
            return normal_explicit(v, sens, phi, masks) + rho * v

    if alpha0 is None:
        alpha = np.zeros(shape, dtype=np.complex128)
    else:
        alpha = np.array(alpha0, dtype=np.complex128, copy=True)
    z = alpha.copy()
    u = np.zeros_like(alpha)
    history = []
    k_freeze = -1
    k = 0
    while k < n_outer:
        alpha = cg(apply_m, alpha, b0 + rho * (z - u), n_cg)
        z_prev = z
        if fixed_shift is not None:
            shift = fixed_shift
        elif k_freeze >= 0:
            shift = block_shift(seed, g, k_freeze, b)
        else:
            shift = block_shift(seed, g, k, b)
        z = llr_prox(alpha + u, tau, shift, b)
        u = u + alpha - z
        rp, rd = admm_residuals(alpha, z, z_prev, u, rho, b0_norm)
        history.append(dict(k=k, shift=shift, r_primal=rp, r_dual=rd, res=max(rp, rd)))
        k += 1
        if replay is not None:
            rk_freeze, rn = replay
            if rk_freeze >= 0 and k - 1 == rk_freeze:
                k_freeze = rk_freeze
            if k >= rn:
                break
            continue
        if tol > 0 and k % check_every == 0:
            res = history[-1]["res"]
            if res <= tol:
                break
            if k_freeze < 0 and k - 1 >= freeze_window:
                if res > (1.0 - freeze_stall) * history[k - 1 - freeze_window]["res"]:
                    k_freeze = k - 1
    return AdmmResult(alpha, z, u, history, k_freeze, k)


# ---------------------------------------------------------------------------
# Post-step (Sec. II-B end; Sec. IV-A post-processing): spatial wavelet
# soft-threshold of each coefficient image, then back-projection (eq. backproj)
# ---------------------------------------------------------------------------


def haar2(x):
    """One level of the orthonormal separable 2D Haar transform over the last two axes:
    (LL, LH, HL, HH), LH differencing along z, HL along y, each half size."""
    a, b = x[..., 0::2, 0::2], x[..., 0::2, 1::2]
    c, d = x[..., 1::2, 0::2], x[..., 1::2, 1::2]
    return (a + b + c + d) / 2, (a - b + c - d) / 2, (a + b - c - d) / 2, (a - b - c + d) / 2


def ihaar2(LL, LH, HL, HH):
    """Inverse of ``haar2``."""
    out = np.empty(LL.shape[:-2] + (2 * LL.shape[-2], 2 * LL.shape[-1]), dtype=np.result_type(LL, 1.0))
    out[..., 0::2, 0::2] = (LL + LH + HL + HH) / 2
    out[..., 0::2, 1::2] = (LL - LH + HL - HH) / 2
    out[..., 1::2, 0::2] = (LL + LH - HL - HH) / 2
    out[..., 1::2, 1::2] = (LL - LH - HL + HH) / 2
    return out


def soft_threshold(c, t):
    """Complex soft threshold: c max(1 - t / |c|, 0)."""
    r = np.abs(c)
    return c * np.where(r > t, 1.0 - t / np.maximum(r, 1e-300), 0.0)


def wavelet_denoise(alpha, levels, thresh):
    """`levels`-level orthonormal 2D Haar transform of every image (last two axes), soft
    threshold of every detail coefficient, inverse; the coarsest approximation is kept."""
    x = np.asarray(alpha, dtype=np.complex128)
    details = []
    for _ in range(levels):
        x, lh, hl, hh = haar2(x)
        details.append(tuple(soft_threshold(d, thresh) for d in (lh, hl, hh)))
    for lh, hl, hh in reversed(details):
        x = ihaar2(x, lh, hl, hh)
    return x


def backproject(alpha, phi_te):
    """Images at chosen echo times, eq. (backproj): x_j = sum_k phi_te[j, k] alpha_k."""
    return np.tensordot(np.asarray(phi_te, dtype=np.float64), np.asarray(alpha, dtype=np.complex128), axes=(1, 0))


# ---------------------------------------------------------------------------
# Readout decoupling (Sec. II-A end; Sec. IV-A, before the PICS reconstruction): a
# 1D unitary inverse DFT along the fully sampled readout turns 3D data into slices
# ---------------------------------------------------------------------------


def readout_ifft(ksp3d):
    """Centred unitary inverse DFT along the last axis of [C, P, Nx] samples (index kx is
    frequency kx - Nx/2, output x is position x - Nx/2), returned as [Nx, C, P]: slice x's
    samples in mask order."""
    k = np.asarray(ksp3d, dtype=np.complex128)
    x = np.fft.fftshift(np.fft.ifft(np.fft.ifftshift(k, axes=-1), axis=-1, norm="ortho"), axes=-1)
    return np.moveaxis(x, -1, 0)


# ---------------------------------------------------------------------------
# FISTA (the paper's solver, Sec. II-A), at a fixed block shift or under the random
# shift schedule of the ADMM z-step
# ---------------------------------------------------------------------------


def lipschitz(sens, psi, v0, n_iter):
    """Largest eigenvalue of A^H A by power iteration from v0: v <- N v / ||v||, and the
    Rayleigh quotient <v, N v> / <v, v> of the last iterate (0 if v0 = 0)."""
    v = np.asarray(v0, dtype=np.complex128)
    L = 0.0
    nv = None
    for j in range(n_iter):
        if j > 0:
            nrm = np.linalg.norm(v)
            v = nv / nrm if nrm > 0 else nv * 0.0
        nv = normal_psi(v, sens, psi)
        vv = np.vdot(v, v).real
        L = np.vdot(v, nv).real / vv if vv > 0 else 0.0
    return L


def fista(samples, sens, phi, masks, lam, b, n_iter, shift=None, step=None, seed=None, g=0, alpha0=None):
    """Proximal gradient with Nesterov momentum (Beck & Teboulle 2009) on eq. (t2shpics).

    The gradient is A^H A x - A^H y and the prox is the blocked LLR threshold
    lambda * step, at the fixed ``shift`` or, with ``seed``, at block_shift(seed, g, k, b)
    in iteration k.  The step is 1/L with L the largest eigenvalue of A^H A (power
    iteration from a random vector when not given).  Momentum: t_0 = 1,
    t_(k+1) = (1 + sqrt(1 + 4 t_k^2)) / 2, y_(k+1) = x_(k+1) + (t_k - 1)/t_(k+1) (x_(k+1) - x_k),
    started at y_0 = x_0 = alpha0 (0 when not given).
    """
    if (shift is None) == (seed is None):
        raise ValueError("give either a fixed shift or a seed")
    sens = np.asarray(sens, dtype=np.complex128)
    phi = np.asarray(phi, dtype=np.float64)
    K = phi.shape[1]
    Ny, Nz = sens.shape[-2:]
    shape = (K, Ny, Nz) if sens.ndim == 3 else (sens.shape[1], K, Ny, Nz)
    psi = space_time_kernel(phi, masks)
    aty = adjoint(samples, sens, phi, masks)
    if step is None:
        v0 = np.random.default_rng(1).standard_normal(shape) + 0j
        step = 1.0 / lipschitz(sens, psi, v0, 101)
    x = np.zeros(shape, dtype=np.complex128) if alpha0 is None else np.array(alpha0, dtype=np.complex128)
    yk = x.copy()
    t = 1.0
    for k in range(n_iter):
        sh = shift if seed is None else block_shift(seed, g, k, b)
        grad = normal_psi(yk, sens, psi) - aty
        x_new = llr_prox(yk - step * grad, lam * step, sh, b)
        t_new = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
        yk = x_new + ((t - 1.0) / t_new) * (x_new - x)
        x, t = x_new, t_new
    return x
