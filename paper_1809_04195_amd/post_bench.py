"""Throughput of the post-step kernels on the 320-slice 256^2 volume (K = 4): the
4-level Haar soft-threshold of every coefficient image (t2s_wavelet_denoise, in place)
and the back-projection onto 3 echo times (t2s_backproject), against the HBM roofline.
Algorithmic bytes: denoise one read and one write of alpha (2 S K N 8); back-projection
one read of alpha and one write of the images (S (K + 3) N 8).

    python -m paper_1809_04195_amd.post_bench
"""

from __future__ import annotations

import json
import sys

import numpy as np

HBM_PEAK_GBS = 8000.0


def main():
    import torch

    from . import Plan, t2s_load_slices

    assert torch.cuda.is_available(), "needs a GPU"
    S, ny, nz, C, Tn, K, nte = 320, 256, 256, 8, 80, 4, 3
    rng = np.random.default_rng(0)
    phi, _ = np.linalg.qr(rng.standard_normal((Tn, K)))
    masks = (rng.random((Tn, ny, nz)) < 0.015).astype(np.uint8)
    P = int(masks.sum())
    plan = Plan(phi.astype(np.float32), [dict(ny=ny, nz=nz, ncoils=C, nslices=S, masks=masks)], lam=0.01, rho=0.1)
    g = torch.Generator(device="cuda").manual_seed(0)
    sens = torch.randn((S, C, ny, nz), dtype=torch.complex64, device="cuda", generator=g)
    sens /= sens.abs().square().sum(1, keepdim=True).sqrt()
    ksp = torch.randn((S, C, P), dtype=torch.complex64, device="cuda", generator=g)
    stream = torch.cuda.current_stream()
    t2s_load_slices(plan.handle, 0, 0, S, sens, ksp, stream)
    del sens, ksp
    a0 = torch.randn((S, K, ny, nz), dtype=torch.complex64, device="cuda", generator=g)
    plan.set_initial(0, 0, a0)
    del a0
    sel = phi[[3, 8, 15]].astype(np.float32)
    out = torch.empty((S, nte, ny, nz), dtype=torch.complex64, device="cuda")
    from . import t2s_backproject

    def timed(fn, reps=10):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    N = ny * nz
    ms_d = timed(lambda: plan.wavelet_denoise(0, 0, S, 4, 0.01, stream))
    ms_b = timed(lambda: t2s_backproject(plan.handle, 0, 0, S, sel, out, stream))
    gb_d = 2.0 * S * K * N * 8 / 1e9
    gb_b = S * (K + nte) * N * 8 / 1e9
    res = dict(workload="vol320_256x256_k4", slices=S,
               wavelet_denoise=dict(levels=4, ms=round(ms_d, 4), alg_gb=round(gb_d, 3), gbs=round(gb_d / ms_d * 1e3, 1),
                                    frac_hbm_peak=round(gb_d / ms_d * 1e3 / HBM_PEAK_GBS, 4)),
               backproject=dict(echo_times=nte, ms=round(ms_b, 4), alg_gb=round(gb_b, 3),
                                gbs=round(gb_b / ms_b * 1e3, 1), frac_hbm_peak=round(gb_b / ms_b * 1e3 / HBM_PEAK_GBS, 4)))
    print(f"[post_bench] denoise {ms_d:.3f} ms, back-projection {ms_b:.3f} ms", file=sys.stderr, flush=True)
    print(json.dumps(res), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
