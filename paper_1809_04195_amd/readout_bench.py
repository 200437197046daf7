"""Throughput of the readout pre-step (t2s_readout_ifft) on the sample arrays of the
two volume workloads, against the HBM roofline: algorithmic bytes = one read and one
write of every complex64 sample (2 x nx x C x P x 8 bytes).

    python -m paper_1809_04195_amd.readout_bench

Shapes: 320-point readout, 8 coils, 80 echoes x 983 samples (256^2 slices at 1.5 %);
512-point readout, 16 coils, 100 echoes x 1475 samples (384^2 slices at 1 %).
Inputs are random (the transform does not depend on the values).
"""

from __future__ import annotations

import json
import sys

HBM_PEAK_GBS = 8000.0
SHAPES = {"vol320_256x256_c8_t80": (320, 8, 80 * 983), "vol512_384x384_c16_t100": (512, 16, 100 * 1475)}


def main():
    import torch

    from . import t2s_readout_ifft

    assert torch.cuda.is_available(), "needs a GPU"
    res = {}
    for name, (nx, C, P) in SHAPES.items():
        g = torch.Generator(device="cuda").manual_seed(0)
        inp = torch.randn((C, P, nx), dtype=torch.complex64, device="cuda", generator=g)
        out = torch.empty((nx, C, P), dtype=torch.complex64, device="cuda")
        for _ in range(3):
            t2s_readout_ifft(inp, out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record()
        for _ in range(reps):
            t2s_readout_ifft(inp, out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gb = 2.0 * nx * C * P * 8 / 1e9
        res[name] = dict(nx=nx, coils=C, samples=P, ms=round(ms, 4), alg_gb=round(gb, 3),
                         gbs=round(gb / ms * 1e3, 1), frac_hbm_peak=round(gb / ms * 1e3 / HBM_PEAK_GBS, 4))
        print(f"[readout_bench] {name}: {ms:.3f} ms, {gb / ms * 1e3:.0f} GB/s", file=sys.stderr, flush=True)
        del inp, out
        torch.cuda.empty_cache()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
