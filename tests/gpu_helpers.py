"""Shared helpers of the GPU parity tests (inputs only; no arithmetic of the method)."""

import numpy as np


def crandn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)


def random_problem(seed, ny, nz, C, T, K, S=1, frac=0.2):
    """Random orthonormal basis, SoS-normalised random coil maps, random masks and samples."""
    rng = np.random.default_rng(seed)
    phi, _ = np.linalg.qr(rng.standard_normal((T, K)))
    phi = phi.astype(np.float32)
    sens = crandn(rng, S, C, ny, nz)
    sens /= np.sqrt((np.abs(sens) ** 2).sum(1, keepdims=True))
    sens = sens.astype(np.complex64)
    masks = (rng.random((T, ny, nz)) < frac).astype(np.uint8)
    P = int(masks.sum())
    ksp = crandn(rng, S, C, P)
    return phi, sens, masks, ksp


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def random_problem_maps(seed, ny, nz, C, M, phi, S=1, frac=0.02):
    """Random problem with M coil-map sets (soft-SENSE): maps [S, C, M, ny, nz] normalised
    so that sum over coils and sets of |S|^2 is 1, random masks and samples for the basis
    phi [T, K]."""
    rng = np.random.default_rng(seed)
    T = phi.shape[0]
    sens = crandn(rng, S, C, M, ny, nz)
    sens /= np.sqrt((np.abs(sens) ** 2).sum((1, 2), keepdims=True))
    sens = sens.astype(np.complex64)
    masks = (rng.random((T, ny, nz)) < frac).astype(np.uint8)
    ksp = crandn(rng, S, C, int(masks.sum()))
    return sens, masks, ksp
