"""FP64 oracle of the warm-start U-Net (test infrastructure only).

TEST INFRASTRUCTURE ONLY: imported by tests/ (and nothing in the product path).

The network maps the zero-filled adjoint b0 = A^H y of a slice, packed as 2K real
channels and divided by s = max |b0|, to the ADMM solution divided by s.  The
paper has no such network (its reconstruction is plain iterative); this is the
warm start of the target workload, with the architecture readings:

* NHWC tensors [B, H, W, C]; 4 levels, base width F: channels F, 2F, 4F, 8F.
* Encoder level l < L-1: conv3x3 + ReLU, conv3x3 + ReLU (its output is the skip),
  2x2 max-pool.  Bottleneck (level L-1): two conv3x3 + ReLU.
* Decoder level l = L-2 .. 0: 2x2 stride-2 transposed conv (up) from the level
  below to c_l channels, concatenated [up, skip] (up first), conv3x3 + ReLU twice.
* Final 1x1 conv to the input channel count, global residual: out = x + net(x).
* conv3x3: out[b,y,x,o] = bias[o] + sum_{kh,kw,i} W[kh,kw,o,i] in[b, y+kh-1, x+kw-1, i]
  (zero outside the image).  up: out[b, 2y+i, 2x+j, o] = bias[o] + sum_c W[i,j,o,c] in[b,y,x,c].
  Max-pool gradient goes to the first maximum of each window (row-major scan).
* Parameters are packed into one flat vector, layer by layer in forward order,
  each layer as W[KH][KW][Cout][Cin] followed by bias[Cout].
* Loss: mean squared error over all output elements.
"""

from __future__ import annotations

import numpy as np


def layer_specs(cin, base=32, levels=4):
    """List of (name, kind, KS, Cin, Cout) in forward order."""
    ch = [base * (2 ** l) for l in range(levels)]
    specs = []
    prev = cin
    for l in range(levels - 1):
        specs.append((f"enc{l}a", "conv", 3, prev, ch[l]))
        specs.append((f"enc{l}b", "conv", 3, ch[l], ch[l]))
        prev = ch[l]
    specs.append(("bota", "conv", 3, prev, ch[-1]))
    specs.append(("botb", "conv", 3, ch[-1], ch[-1]))
    below = ch[-1]
    for l in range(levels - 2, -1, -1):
        specs.append((f"up{l}", "up", 2, below, ch[l]))
        specs.append((f"dec{l}a", "conv", 3, 2 * ch[l], ch[l]))
        specs.append((f"dec{l}b", "conv", 3, ch[l], ch[l]))
        below = ch[l]
    specs.append(("final", "conv", 1, ch[0], cin))
    return specs


def param_count(cin, base=32, levels=4):
    return sum(k * k * ci * co + co for _, _, k, ci, co in layer_specs(cin, base, levels))


def unpack(params, cin, base=32, levels=4):
    out, off = {}, 0
    for name, kind, k, ci, co in layer_specs(cin, base, levels):
        n = k * k * co * ci
        W = params[off:off + n].reshape(k, k, co, ci)
        off += n
        b = params[off:off + co]
        off += co
        out[name] = (W, b)
    assert off == params.size
    return out


def init_params(cin, base=32, levels=4, seed=0, final_scale=0.1):
    """He-normal weights, zero biases; the final 1x1 layer scaled down so the
    untrained network is close to the identity (residual)."""
    rng = np.random.default_rng(seed)
    chunks = []
    for name, kind, k, ci, co in layer_specs(cin, base, levels):
        fan_in = (k * k * ci) if kind == "conv" else ci
        W = rng.standard_normal((k, k, co, ci)) * np.sqrt(2.0 / fan_in)
        if name == "final":
            W *= final_scale
        chunks += [W.reshape(-1), np.zeros(co)]
    return np.concatenate(chunks).astype(np.float32)


# ---------------------------------------------------------------------------
# primitives (FP64)
# ---------------------------------------------------------------------------


def conv(x, W, b, relu):
    B, H, Wd, Ci = x.shape
    k = W.shape[0]
    p = k // 2
    xp = np.pad(x, ((0, 0), (p, p), (p, p), (0, 0)))
    out = np.zeros((B, H, Wd, W.shape[2]))
    for kh in range(k):
        for kw in range(k):
            out += np.einsum("byxi,oi->byxo", xp[:, kh:kh + H, kw:kw + Wd, :], W[kh, kw])
    out += b
    return np.maximum(out, 0.0) if relu else out


def conv_backward(x, W, out, dout, relu):
    """Returns (dx, dW, db) of conv; `out` is the forward output (post-ReLU)."""
    if relu:
        dout = dout * (out > 0)
    B, H, Wd, Ci = x.shape
    k = W.shape[0]
    p = k // 2
    xp = np.pad(x, ((0, 0), (p, p), (p, p), (0, 0)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for kh in range(k):
        for kw in range(k):
            dW[kh, kw] = np.einsum("byxo,byxi->oi", dout, xp[:, kh:kh + H, kw:kw + Wd, :])
            dxp[:, kh:kh + H, kw:kw + Wd, :] += np.einsum("byxo,oi->byxi", dout, W[kh, kw])
    dx = dxp[:, p:p + H, p:p + Wd, :]
    return dx, dW, dout.sum(axis=(0, 1, 2))


def up(x, W, b):
    B, H, Wd, Ci = x.shape
    out = np.zeros((B, 2 * H, 2 * Wd, W.shape[2]))
    for i in range(2):
        for j in range(2):
            out[:, i::2, j::2, :] = np.einsum("byxc,oc->byxo", x, W[i, j]) + b
    return out


def up_backward(x, W, dout):
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for i in range(2):
        for j in range(2):
            g = dout[:, i::2, j::2, :]
            dW[i, j] = np.einsum("byxo,byxc->oc", g, x)
            dx += np.einsum("byxo,oc->byxc", g, W[i, j])
    return dx, dW, dout.sum(axis=(0, 1, 2))


def pool(x):
    B, H, Wd, C = x.shape
    v = x.reshape(B, H // 2, 2, Wd // 2, 2, C)
    return v.max(axis=(2, 4))


def pool_backward(x, dout):
    B, H, Wd, C = x.shape
    win = x.reshape(B, H // 2, 2, Wd // 2, 2, C).transpose(0, 1, 3, 5, 2, 4).reshape(B, H // 2, Wd // 2, C, 4)
    arg = win.argmax(axis=-1)                    # first maximum in row-major window order
    onehot = (np.arange(4) == arg[..., None]).astype(x.dtype)
    g = onehot * dout[..., None]
    return g.reshape(B, H // 2, Wd // 2, C, 2, 2).transpose(0, 1, 4, 2, 5, 3).reshape(B, H, Wd, C)


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------


def forward(params, x, base=32, levels=4):
    """out = x + net(x); returns (out, cache)."""
    x = np.asarray(x, dtype=np.float64)
    cin = x.shape[-1]
    P = {k: (W.astype(np.float64), b.astype(np.float64)) for k, (W, b) in unpack(np.asarray(params), cin, base, levels).items()}
    cache = {"x": x}
    h = x
    skips = []
    for l in range(levels - 1):
        a = conv(h, *P[f"enc{l}a"], True)
        e = conv(a, *P[f"enc{l}b"], True)
        cache[f"enc{l}a_in"], cache[f"enc{l}a"] = h, a
        cache[f"enc{l}b"] = e
        skips.append(e)
        h = pool(e)
        cache[f"pool{l}"] = h
    a = conv(h, *P["bota"], True)
    bt = conv(a, *P["botb"], True)
    cache["bota_in"], cache["bota"], cache["botb"] = h, a, bt
    h = bt
    for l in range(levels - 2, -1, -1):
        u = up(h, *P[f"up{l}"])
        cat = np.concatenate([u, skips[l]], axis=-1)
        a = conv(cat, *P[f"dec{l}a"], True)
        d = conv(a, *P[f"dec{l}b"], True)
        cache[f"up{l}_in"], cache[f"cat{l}"], cache[f"dec{l}a"], cache[f"dec{l}b"] = h, cat, a, d
        h = d
    y = conv(h, *P["final"], False)
    cache["final_in"] = h
    return x + y, cache


def backward(params, cache, dout, base=32, levels=4):
    """Gradient of a scalar loss w.r.t. the packed parameters, given dL/dout."""
    x = cache["x"]
    cin = x.shape[-1]
    P = {k: (W.astype(np.float64), b.astype(np.float64)) for k, (W, b) in unpack(np.asarray(params), cin, base, levels).items()}
    G = {}
    dh, G["final_W"], G["final_b"] = conv_backward(cache["final_in"], P["final"][0], None, dout, False)
    dskip = {}
    ch = [base * (2 ** l) for l in range(levels)]
    for l in range(levels - 1):
        dh, G[f"dec{l}b_W"], G[f"dec{l}b_b"] = conv_backward(cache[f"dec{l}a"], P[f"dec{l}b"][0], cache[f"dec{l}b"], dh, True)
        dcat, G[f"dec{l}a_W"], G[f"dec{l}a_b"] = conv_backward(cache[f"cat{l}"], P[f"dec{l}a"][0], cache[f"dec{l}a"], dh, True)
        du, dskip[l] = dcat[..., :ch[l]], dcat[..., ch[l]:]
        dh, G[f"up{l}_W"], G[f"up{l}_b"] = up_backward(cache[f"up{l}_in"], P[f"up{l}"][0], du)
    dh, G["botb_W"], G["botb_b"] = conv_backward(cache["bota"], P["botb"][0], cache["botb"], dh, True)
    dh, G["bota_W"], G["bota_b"] = conv_backward(cache["bota_in"], P["bota"][0], cache["bota"], dh, True)
    for l in range(levels - 2, -1, -1):
        de = pool_backward(cache[f"enc{l}b"], dh) + dskip[l]
        dh, G[f"enc{l}b_W"], G[f"enc{l}b_b"] = conv_backward(cache[f"enc{l}a"], P[f"enc{l}b"][0], cache[f"enc{l}b"], de, True)
        dh, G[f"enc{l}a_W"], G[f"enc{l}a_b"] = conv_backward(cache[f"enc{l}a_in"], P[f"enc{l}a"][0], cache[f"enc{l}a"], dh, True)
    flat = []
    for name, kind, k, ci, co in layer_specs(cin, base, levels):
        flat += [G[f"{name}_W"].reshape(-1), G[f"{name}_b"]]
    return np.concatenate(flat)


def mse(out, target):
    d = out - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def loss_and_grad(params, x, target, base=32, levels=4):
    out, cache = forward(params, x, base, levels)
    loss, dout = mse(out, np.asarray(target, dtype=np.float64))
    return loss, backward(params, cache, dout, base, levels)


# ---------------------------------------------------------------------------
# complex coefficient images <-> normalised real channels
# ---------------------------------------------------------------------------


def pack(alpha, scale):
    """complex [K, H, W] / scale -> real [H, W, 2K] ordered (Re a_0, Im a_0, Re a_1, ...)."""
    a = np.asarray(alpha) / scale
    return np.stack([a.real, a.imag], axis=-1).transpose(1, 2, 0, 3).reshape(a.shape[1], a.shape[2], -1)


def unpack_channels(x, scale):
    H, W, C = x.shape
    v = x.reshape(H, W, C // 2, 2).transpose(2, 0, 1, 3)
    return scale * (v[..., 0] + 1j * v[..., 1])


# ---------------------------------------------------------------------------
# optimiser: Adam (Kingma & Ba, "Adam: a method for stochastic optimization",
# ICLR 2015, Algorithm 1), FP64
# ---------------------------------------------------------------------------


def adam_step(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Update number t >= 1 of the parameters w with gradient g from moments (m, v):
    m <- beta1 m + (1 - beta1) g,  v <- beta2 v + (1 - beta2) g^2,
    m_hat = m / (1 - beta1^t),  v_hat = v / (1 - beta2^t),
    w <- w - lr m_hat / (sqrt(v_hat) + eps).
    Returns (w, m, v)."""
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return w - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
