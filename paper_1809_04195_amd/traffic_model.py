"""Algorithmic HBM bytes of the solver kernels (what each kernel must move, per slice),
the figures the measured launch times are divided by to report bandwidth against
the HBM roofline."""

from __future__ import annotations


def alg_bytes_per_slice(kind, ny, nz, C, K, n_cg):
    """Bytes one slice costs one launch of kernel family `kind` (pass_a averaged over the
    CG steps of an outer iteration; None for kernels without a byte model)."""
    N = ny * nz
    c8 = 8.0 * N
    if kind == "pass_a":       # read r (+ p), S; write p, C K transformed rows
        first = c8 * (2 * K + C + C * K)
        rest = c8 * (3 * K + C + C * K)
        return (first + (n_cg - 1) * rest) / n_cg
    if kind == "pass_b":       # read + write the C K intermediate, read Psi (upper triangle, fp32)
        return c8 * 2 * C * K + 4.0 * N * K * (K + 1) / 2
    if kind == "pass_c":       # read C K intermediate, S, p, x, r; write x, r (CG update fused)
        return c8 * (C * K + C + 5 * K)
    if kind == "llr_admm":     # read alpha, u, z, r; write z, u, r
        return c8 * 7 * K
    if kind == "load_adjoint":
        return None
    raise KeyError(kind)


def bytes_per_outer(ny, nz, C, K, n_cg):
    """Algorithmic bytes of one ADMM outer iteration of one slice."""
    return (n_cg * sum(alg_bytes_per_slice(k, ny, nz, C, K, n_cg) for k in ("pass_a", "pass_b", "pass_c"))
            + alg_bytes_per_slice("llr_admm", ny, nz, C, K, n_cg))
