"""Throughput of the warm-start network's kernels (bf16 matrix cores): inference
slices/s and training slice-steps/s on synthetic inputs, with the algorithmic
FLOP rate against the dense bf16 matrix-core peak of one MI355X.

    python -m paper_1809_04195_amd.unet_bench [--K 4 --size 256 --batch 16]

Algorithmic FLOPs count the network's true channel counts (the kernels pad the
2K input and output channels to 16); a training step counts 3 forward passes
(forward, data gradient, weight gradient).
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import UNet

BF16_DENSE_PEAK_TFLOPS = 2500.0


def forward_flops(cin, H, W, base=32, levels=4):
    """2 x multiply-adds of one forward pass on one H x W slice: per level two 3x3
    convolutions, 2x2 stride-2 transposed convolutions on the way up into a [up, skip]
    concatenation, final 1x1 convolution."""
    ch = [base * 2 ** l for l in range(levels)]
    px = [H * W // 4 ** l for l in range(levels)]
    macs, prev = 0, cin
    for l in range(levels):
        macs += px[l] * 9 * (prev * ch[l] + ch[l] * ch[l])
        prev = ch[l]
    for l in range(levels - 2, -1, -1):
        macs += px[l] * ch[l + 1] * ch[l]                       # transposed conv: 1 tap per output pixel
        macs += px[l] * 9 * (2 * ch[l] * ch[l] + ch[l] * ch[l])
    macs += px[0] * ch[0] * cin
    return 2 * macs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--K", type=int, default=4)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    args = ap.parse_args()

    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    K, H, B = args.K, args.size, args.batch
    net = UNet(K, 32, 4, max_batch=B, H=H, W=H)
    net.set_params(net.init_params(0))
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn((B, K, H, H), dtype=torch.complex64, device="cuda", generator=g)
    t = x + 0.1 * torch.randn((B, K, H, H), dtype=torch.complex64, device="cuda", generator=g)
    out = torch.empty_like(x)
    fl = forward_flops(2 * K, H, H)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.iters):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.iters

    t0 = time.perf_counter()
    ms_f = timed(lambda: net.forward(x, out))
    print(f"[unet_bench] forward {ms_f:.3f} ms per batch of {B}", file=sys.stderr, flush=True)
    ms_t = timed(lambda: net.train_step(x, t, 1e-4))
    print(f"[unet_bench] train step {ms_t:.3f} ms per batch of {B}", file=sys.stderr, flush=True)
    res = dict(network=f"U-Net 4 levels base 32, {2 * K} channels in/out, {H}x{H}", batch=B,
               forward_gflop_per_slice=round(fl / 1e9, 3),
               forward=dict(ms_per_batch=round(ms_f, 4), slices_per_s=round(B / ms_f * 1e3, 1),
                            tflops=round(fl * B / ms_f / 1e9, 1),
                            frac_bf16_peak=round(fl * B / ms_f / 1e9 / BF16_DENSE_PEAK_TFLOPS, 4)),
               train=dict(ms_per_batch=round(ms_t, 4), slice_steps_per_s=round(B / ms_t * 1e3, 1),
                          tflops=round(3 * fl * B / ms_t / 1e9, 1),
                          frac_bf16_peak=round(3 * fl * B / ms_t / 1e9 / BF16_DENSE_PEAK_TFLOPS, 4)),
               peak_tflops=BF16_DENSE_PEAK_TFLOPS, wall_s=round(time.perf_counter() - t0, 2))
    print(json.dumps(res), flush=True)
    net.close()


if __name__ == "__main__":
    np.random.seed(0)
    main()
