"""GPU checks of the warm-start network kernels against the FP64 oracle.

BF16 activations and weights with FP32 accumulation: per-tensor relative L2 within
2e-2 of the FP64 result and cosine similarity >= 0.999 (gradients: see below).
"""

import sys

import numpy as np
import pytest

import paper_1809_04195_amd as T
from oracle import unet as U

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu(gpu):
    return gpu


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def bf16_round(a):
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32)


def test_mfma_lane_layout():
    rng = np.random.default_rng(0)
    A = rng.integers(-8, 9, (16, 16)).astype(np.float32) / 8
    B = rng.integers(-8, 9, (16, 16)).astype(np.float32) / 4
    D = T.t2s_unet_mfma_probe(A, B)
    assert np.array_equal(D, (A.astype(np.float64) @ B).astype(np.float32))


def test_mfma32_lane_layout():
    """The 32-deep product the convolution kernels use: exact on small dyadic values."""
    rng = np.random.default_rng(1)
    A = rng.integers(-8, 9, (16, 32)).astype(np.float32) / 8
    B = rng.integers(-8, 9, (32, 16)).astype(np.float32) / 4
    D = T.t2s_unet_mfma_probe32(A, B)
    assert np.array_equal(D, (A.astype(np.float64) @ B).astype(np.float32))


def _tiny(seed, K=2, base=16, levels=3, H=16, W=16, B=2):
    rng = np.random.default_rng(seed)
    params = U.init_params(2 * K, base, levels, seed=seed, final_scale=1.0)
    params = params + 0.02 * rng.standard_normal(params.size).astype(np.float32)
    x = rng.standard_normal((B, H, W, 2 * K)).astype(np.float32)
    t = rng.standard_normal((B, H, W, 2 * K)).astype(np.float32)
    return params, x, t


def cos(a, b):
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))


def test_forward_matches_oracle():
    import torch
    K, base, levels, H, W, B = 2, 16, 3, 16, 16, 2
    params, _, _ = _tiny(1, K, base, levels, H, W, B)
    rng = np.random.default_rng(3)
    b0 = (rng.standard_normal((B, K, H, W)) + 1j * rng.standard_normal((B, K, H, W))).astype(np.complex64)
    net = T.UNet(K, base, levels, max_batch=B, H=H, W=W)
    net.set_params(params)
    d_in = torch.from_numpy(b0).cuda()
    d_out = torch.empty_like(d_in)
    net.forward(d_in, d_out)
    torch.cuda.synchronize()
    got = d_out.cpu().numpy()
    for s in range(B):
        scale = np.abs(b0[s]).max()
        x = U.pack(b0[s].astype(np.complex128), scale)[None]
        out, _ = U.forward(params.astype(np.float64), x, base, levels)
        ref_net = out[0] - x[0]
        got_net = U.pack(got[s].astype(np.complex128), scale) - x[0]
        e = np.linalg.norm(got_net - ref_net) / np.linalg.norm(ref_net)
        c = cos(got_net.ravel(), ref_net.ravel())
        _say(f"  slice {s}: net(x) rel L2 {e:.3e} cosine {c:.6f}")
        assert e < 2e-2 and c > 0.999
    # an all-zero slice (no data) maps to an all-zero start; the other slice of the
    # batch is unchanged
    d_in[1] = 0
    d_out2 = torch.empty_like(d_in)
    net.forward(d_in, d_out2)
    torch.cuda.synchronize()
    assert not d_out2[1].any()
    assert torch.equal(d_out2[0], d_out[0])
    net.close()


def test_gradient_matches_oracle():
    K, base, levels, H, W, B = 2, 16, 3, 16, 16, 2
    params, x, t = _tiny(2, K, base, levels, H, W, B)
    net = T.UNet(K, base, levels, max_batch=B, H=H, W=W)
    net.set_params(params)
    loss, g = net.loss_grad(x, t)
    rloss, rg = U.loss_and_grad(params.astype(np.float64), x, t, base, levels)
    _say(f"  loss gpu {loss:.6f} oracle {rloss:.6f}")
    assert abs(loss - rloss) < 2e-2 * rloss
    off = 0
    worst = []
    for name, kind, k, ci, co in U.layer_specs(2 * K, base, levels):
        for part, n in (("W", k * k * ci * co), ("b", co)):
            a, b = g[off:off + n].astype(np.float64), rg[off:off + n]
            off += n
            e = np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-30)
            c = cos(a, b)
            worst.append((e, c, name + part))
            _say(f"  {name}.{part}: rel L2 {e:.3e} cosine {c:.5f}")
    # whole-vector agreement, and every tensor pointing the same way
    e_all = np.linalg.norm(g - rg) / np.linalg.norm(rg)
    assert e_all < 3e-2, e_all
    assert min(c for _, c, _ in worst) > 0.995
    assert cos(g.astype(np.float64), rg) > 0.999
    net.close()


def test_training_reduces_loss():
    import torch
    K, base, levels, H, W, B = 2, 16, 3, 32, 32, 4
    rng = np.random.default_rng(5)
    params = U.init_params(2 * K, base, levels, seed=5)
    net = T.UNet(K, base, levels, max_batch=B, H=H, W=W)
    net.set_params(params)
    # target: a smoothed, rescaled copy of the input (learnable by a small conv net)
    b0 = (rng.standard_normal((B, K, H, W)) + 1j * rng.standard_normal((B, K, H, W))).astype(np.complex64)
    sm = 0.25 * (b0 + np.roll(b0, 1, 2) + np.roll(b0, 1, 3) + np.roll(b0, (1, 1), (2, 3)))
    tgt = (1.5 * sm).astype(np.complex64)
    db0 = torch.from_numpy(b0).cuda()
    dt = torch.from_numpy(tgt).cuda()
    losses = [net.train_step(db0, dt, 3e-3, want_loss=True) for _ in range(60)]
    _say(f"  loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.3 * losses[0]
    assert np.all(np.isfinite(net.get_params()))
    net.close()


def test_adam_matches_oracle():
    """The optimiser step of the training path (t2s_unet_adam_apply: the same update
    t2s_unet_train_step applies after its backward pass) against the FP64 Adam oracle,
    over three steps with seeded gradients spanning eight decades, moments included."""
    K, base, levels, H, W = 2, 16, 3, 16, 16
    rng = np.random.default_rng(11)
    p0 = U.init_params(2 * K, base, levels, seed=11, final_scale=1.0)
    net = T.UNet(K, base, levels, max_batch=1, H=H, W=W)
    net.set_params(p0)
    w = p0.astype(np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    for t, lr in ((1, 1e-3), (2, 1e-3), (3, 3e-4)):
        g = (rng.standard_normal(p0.size) * 10.0 ** rng.uniform(-5, 3, p0.size)).astype(np.float32)
        net.adam_apply(g, lr)
        w, m, v = U.adam_step(w, g.astype(np.float64), m, v, t, lr)
        gw = net.get_params().astype(np.float64)
        gm, gv, step = net.adam_state()
        ew = np.abs(gw - w).max() / lr
        em = np.abs(gm - m).max() / np.abs(m).max()
        ev = np.abs(gv - v).max() / np.abs(v).max()
        _say(f"  step {t}: |dw| / lr {ew:.2e}, m {em:.2e}, v {ev:.2e}")
        assert step == t
        assert np.all(np.abs(gw - w) <= 2.0 ** -22 * np.abs(w) + 1e-4 * lr)
        np.testing.assert_allclose(gm, m, rtol=1e-5, atol=1e-7 * np.abs(m).max())
        np.testing.assert_allclose(gv, v, rtol=1e-5, atol=1e-7 * np.abs(v).max())
    net.close()


def test_train_step_is_backward_then_adam():
    """One t2s_unet_train_step from fresh optimiser state equals the oracle's gradient
    followed by the oracle's first Adam step: every weight moves by lr g / (|g| + eps),
    i.e. by ~lr against the sign of its gradient.  bf16 gradients may flip the sign of
    gradients that are small next to their tensor: all but 0.1 % of the weights whose
    gradient exceeds 0.3 times its tensor's root mean square must move exactly as the
    oracle's (the Adam kernel itself is checked exactly by test_adam_matches_oracle)."""
    import torch
    K, base, levels, H, W, B = 2, 16, 3, 16, 16, 2
    rng = np.random.default_rng(12)
    p0 = U.init_params(2 * K, base, levels, seed=12, final_scale=1.0)
    p0 = p0 + 0.02 * rng.standard_normal(p0.size).astype(np.float32)
    b0 = (rng.standard_normal((B, K, H, W)) + 1j * rng.standard_normal((B, K, H, W))).astype(np.complex64)
    tgt = (0.7 * b0 + 0.1 * np.roll(b0, 1, 2)).astype(np.complex64)
    net = T.UNet(K, base, levels, max_batch=B, H=H, W=W)
    net.set_params(p0)
    lr = 1e-3
    net.train_step(torch.from_numpy(b0).cuda(), torch.from_numpy(tgt).cuda(), lr)
    dw = net.get_params().astype(np.float64) - p0
    x = np.stack([U.pack(b0[s].astype(np.complex128), np.abs(b0[s]).max()) for s in range(B)])
    t = np.stack([U.pack(tgt[s].astype(np.complex128), np.abs(b0[s]).max()) for s in range(B)])
    _, g = U.loss_and_grad(p0.astype(np.float64), x, t, base, levels)
    w1, _, _ = U.adam_step(p0.astype(np.float64), g, 0.0, 0.0, 1, lr)
    dref = w1 - p0
    # large gradient: at least 0.3 times the root mean square of its tensor's gradient
    big = np.zeros(g.size, dtype=bool)
    off = 0
    for name, kind, k, ci, co in U.layer_specs(2 * K, base, levels):
        for n in (k * k * ci * co, co):
            seg = g[off:off + n]
            big[off:off + n] = np.abs(seg) > 0.3 * np.sqrt(np.mean(seg * seg))
            off += n
    agree = np.mean(np.sign(dw) == np.sign(dref))
    bad = np.abs(dw[big] - dref[big]) > 2e-3 * lr + 2.0 ** -23 * np.abs(p0[big])
    _say(f"  {big.mean():.3f} of the weights have large gradients ({bad.sum()} of them moved differently); "
         f"sign agreement over all weights {agree:.4f}")
    assert np.all(np.abs(dw) <= lr * (1 + 1e-3))
    assert bad.sum() <= 1e-3 * big.sum()
    assert agree > 0.97
    net.close()


def test_forward_matches_oracle_deployed_architecture():
    """The deployed network (4 levels, 32 base filters, 2K = 8 channels) on a 256 x 256
    slice against the FP64 oracle."""
    import torch
    K, base, levels, H, W = 4, 32, 4, 256, 256
    rng = np.random.default_rng(13)
    params = U.init_params(2 * K, base, levels, seed=13, final_scale=1.0)
    params = params + 0.01 * rng.standard_normal(params.size).astype(np.float32)
    yy, xx = np.mgrid[0:H, 0:W] / H
    smooth = np.exp(-((yy - 0.5) ** 2 + (xx - 0.45) ** 2) / 0.05)
    b0 = (smooth[None] * (1 + 0.3 * rng.standard_normal((K, H, W)))
          + 0.2j * smooth[None] * rng.standard_normal((K, H, W))).astype(np.complex64)[None]
    net = T.UNet(K, base, levels, max_batch=1, H=H, W=W)
    net.set_params(params)
    d_in = torch.from_numpy(b0).cuda()
    d_out = torch.empty_like(d_in)
    net.forward(d_in, d_out)
    torch.cuda.synchronize()
    got = d_out.cpu().numpy()[0]
    scale = np.abs(b0[0]).max()
    x = U.pack(b0[0].astype(np.complex128), scale)[None]
    out, _ = U.forward(params.astype(np.float64), x, base, levels)
    ref_net = out[0] - x[0]
    got_net = U.pack(got.astype(np.complex128), scale) - x[0]
    e = np.linalg.norm(got_net - ref_net) / np.linalg.norm(ref_net)
    c = cos(got_net.ravel(), ref_net.ravel())
    _say(f"  256x256, 4 levels, base 32: net(x) rel L2 {e:.3e} cosine {c:.6f}")
    assert e < 2e-2 and c > 0.999
    net.close()
