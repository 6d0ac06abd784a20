"""FP64 oracle for the learned prior -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of the
benchmark may import this module.  It never imports the product.

The paper's section on data-driven methods (its learned-reconstruction
discussion) only says that trained networks call the projection operators;
the denoiser itself is a builder's choice, defined here and used
plug-and-play inside CGLS:

* a 3-D residual U-Net with 4 levels of (16, 32, 64, 128) channels; per
  level two [3x3x3 convolution, zero padding 1, + bias, ReLU]; 2x2x2 average
  pooling down; 2x2x2 stride-2 transposed convolution (+ bias, no ReLU) up;
  skip connections by channel concatenation (upsampled channels first);
  a 1x1x1 head to one channel; output = input + head;
* BF16 weights and activations (round to nearest, ties to even) with
  accumulation in high precision; FP32 master weights; MSE loss; Adam.

Tensors are channels-last: activations ``[N, D, H, W, C]``; 3x3x3 weights
``[Cout, 27, Cin]`` with tap t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1) reading the
input at (z + dz, y + dy, x + dx); transposed-convolution weights
``[Cout, 8, Cin]`` with sub-position s = 4 a + 2 b + c writing output voxel
(2z + a, 2y + b, 2x + c).

Every operator is written from its definition (sums over taps with numpy
matrix products as the only library step); the backward passes are the
definitions of the adjoints.  With ``rounding=False`` the network is plain
FP64, which the tests pin to ``torch`` autograd on the CPU.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Tuple

import numpy as np

import synth

CHANNELS = (16, 32, 64, 128)
TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
SUBPOS = [(a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)]


# ----------------------------------------------------------- rounding
def bf16(a) -> np.ndarray:
    """Round to the nearest BF16 value (8 significant bits), ties to even,
    from the exact value: a = f 2^e with f in [0.5, 1) becomes
    rint(256 f) 2^(e - 8)."""
    a = np.asarray(a, dtype=np.float64)
    f, e = np.frexp(a)
    return np.ldexp(np.rint(f * 256.0), e - 8)


def _q(a, rounding: bool):
    return bf16(a) if rounding else np.asarray(a, dtype=np.float64)


# --------------------------------------------------- 3x3x3 convolution
def _pad(x):
    return np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))


def conv3(x, w, b=None) -> np.ndarray:
    """y[v, co] = b[co] + sum_t sum_ci x[v + t, ci] w[co, t, ci], zero outside."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n, d, h, wd, _ = x.shape
    xp = _pad(x)
    y = np.zeros((n, d, h, wd, w.shape[0]))
    for t, (dz, dy, dx) in enumerate(TAPS):
        y += xp[:, 1 + dz:1 + dz + d, 1 + dy:1 + dy + h, 1 + dx:1 + dx + wd, :] @ w[:, t, :].T
    if b is not None:
        y += np.asarray(b, dtype=np.float64)
    return y


def conv3_dgrad(g, w) -> np.ndarray:
    """Adjoint of conv3 in x: dx[u, ci] = sum_t sum_co g[u - t, co] w[co, t, ci]."""
    g = np.asarray(g, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n, d, h, wd, _ = g.shape
    gp = _pad(g)
    dx_ = np.zeros((n, d, h, wd, w.shape[2]))
    for t, (dz, dy, dx) in enumerate(TAPS):
        dx_ += gp[:, 1 - dz:1 - dz + d, 1 - dy:1 - dy + h, 1 - dx:1 - dx + wd, :] @ w[:, t, :]
    return dx_


def conv3_wgrad(x, g) -> Tuple[np.ndarray, np.ndarray]:
    """dw[co, t, ci] = sum_v g[v, co] x[v + t, ci]; db[co] = sum_v g[v, co]."""
    x = np.asarray(x, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    n, d, h, wd, cin = x.shape
    cout = g.shape[-1]
    xp = _pad(x)
    gm = g.reshape(-1, cout)
    dw = np.zeros((cout, 27, cin))
    for t, (dz, dy, dx) in enumerate(TAPS):
        xs = xp[:, 1 + dz:1 + dz + d, 1 + dy:1 + dy + h, 1 + dx:1 + dx + wd, :].reshape(-1, cin)
        dw[:, t, :] = gm.T @ xs
    return dw, gm.sum(axis=0)


# ------------------------------------------------ pooling / upsampling
def pool2(x) -> np.ndarray:
    """2x2x2 average pooling (even sizes)."""
    x = np.asarray(x, dtype=np.float64)
    n, d, h, w, c = x.shape
    return x.reshape(n, d // 2, 2, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4, 6))


def pool2_adjoint(g) -> np.ndarray:
    """Adjoint of pool2: every fine voxel gets its parent's value / 8."""
    g = np.asarray(g, dtype=np.float64) / 8.0
    return g.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def up2(x, w, b=None) -> np.ndarray:
    """Stride-2 2x2x2 transposed convolution:
    y[2v + s, co] = b[co] + sum_ci x[v, ci] w[co, s, ci]."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n, d, h, wd, _ = x.shape
    y = np.zeros((n, 2 * d, 2 * h, 2 * wd, w.shape[0]))
    for s, (a, bb, c) in enumerate(SUBPOS):
        y[:, a::2, bb::2, c::2, :] = x @ w[:, s, :].T
    if b is not None:
        y += np.asarray(b, dtype=np.float64)
    return y


def up2_dgrad(g, w) -> np.ndarray:
    """Adjoint of up2 in x: dx[v, ci] = sum_s sum_co g[2v + s, co] w[co, s, ci]."""
    g = np.asarray(g, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n, d2, h2, w2, _ = g.shape
    dx = np.zeros((n, d2 // 2, h2 // 2, w2 // 2, w.shape[2]))
    for s, (a, bb, c) in enumerate(SUBPOS):
        dx += g[:, a::2, bb::2, c::2, :] @ w[:, s, :]
    return dx


def up2_wgrad(x, g) -> Tuple[np.ndarray, np.ndarray]:
    """dw[co, s, ci] = sum_v g[2v + s, co] x[v, ci]; db[co] = sum g[., co]."""
    x = np.asarray(x, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    cin, cout = x.shape[-1], g.shape[-1]
    xm = x.reshape(-1, cin)
    dw = np.zeros((cout, 8, cin))
    for s, (a, bb, c) in enumerate(SUBPOS):
        dw[:, s, :] = g[:, a::2, bb::2, c::2, :].reshape(-1, cout).T @ xm
    return dw, g.reshape(-1, cout).sum(axis=0)


# ------------------------------------------------------------ network
def layer_shapes(channels=CHANNELS) -> List[Tuple[str, str, Tuple[int, ...]]]:
    """(name, kind, weight shape) for every layer, in forward order.
    kind: 'conv3' (3x3x3), 'up2' (transposed 2x2x2), 'head' (1x1x1)."""
    c = channels
    out = []
    cin = 1
    for lvl, ch in enumerate(c):
        out.append((f"enc{lvl}a", "conv3", (ch, 27, cin)))
        out.append((f"enc{lvl}b", "conv3", (ch, 27, ch)))
        cin = ch
    for lvl in range(len(c) - 2, -1, -1):
        out.append((f"up{lvl}", "up2", (c[lvl], 8, c[lvl + 1])))
        out.append((f"dec{lvl}a", "conv3", (c[lvl], 27, 2 * c[lvl])))
        out.append((f"dec{lvl}b", "conv3", (c[lvl], 27, c[lvl])))
    out.append(("head", "head", (1, 1, c[0])))
    return out


def init_params(seed: int, channels=CHANNELS) -> Dict[str, np.ndarray]:
    """He-normal weights (std sqrt(2 / fan-in), fan-in 27 Cin for 3x3x3 and
    Cin for the transposed convolutions; the head 0.1 / sqrt(Cin)) drawn by
    the shared seeded generator in layer order; zero biases."""
    shapes = layer_shapes(channels)
    specs = []
    for name, kind, shp in shapes:
        fan = shp[1] * shp[2] if kind == "conv3" else shp[2]
        specs.append((shp, math.sqrt(2.0 / fan) if kind != "head" else 0.1 / math.sqrt(fan)))
    ws = synth.normal_weights(seed, specs)
    p = {}
    for (name, _, shp), w in zip(shapes, ws):
        p[name + ".w"] = w.astype(np.float64)
        p[name + ".b"] = np.zeros(shp[0])
    return p


def param_count(channels=CHANNELS) -> int:
    return sum(int(np.prod(s)) + s[0] for _, _, s in layer_shapes(channels))


def forward(params, x_in, rounding: bool = True, channels=CHANNELS):
    """D(x) for x_in [N, D, H, W] (FP32 values); D, H, W divisible by 8.

    Stored tensors (all BF16 when rounding): the rounded input x0, every
    conv output after bias and ReLU, every pool output, every up2 output
    after bias.  The head is computed from the last activation and BF16
    head weights and added to the unrounded input.
    Returns (output [N, D, H, W], cache for backward)."""
    q = lambda a: _q(a, rounding)
    W = {k: (q(v) if k.endswith(".w") else np.asarray(v, dtype=np.float64)) for k, v in params.items()}
    nl = len(channels)
    x_in = np.asarray(x_in, dtype=np.float64)
    c = {"x_in": x_in}
    h = q(x_in[..., None])
    c["x0"] = h
    skips = []
    for lvl in range(nl):
        a = q(np.maximum(conv3(h, W[f"enc{lvl}a.w"], W[f"enc{lvl}a.b"]), 0.0))
        c[f"enc{lvl}a"] = a
        h = q(np.maximum(conv3(a, W[f"enc{lvl}b.w"], W[f"enc{lvl}b.b"]), 0.0))
        c[f"enc{lvl}b"] = h
        if lvl < nl - 1:
            skips.append(h)
            h = q(pool2(h))
            c[f"pool{lvl + 1}"] = h
    for lvl in range(nl - 2, -1, -1):
        u = q(up2(h, W[f"up{lvl}.w"], W[f"up{lvl}.b"]))
        c[f"up{lvl}"] = u
        cat = np.concatenate([u, skips[lvl]], axis=-1)
        a = q(np.maximum(conv3(cat, W[f"dec{lvl}a.w"], W[f"dec{lvl}a.b"]), 0.0))
        c[f"dec{lvl}a"] = a
        h = q(np.maximum(conv3(a, W[f"dec{lvl}b.w"], W[f"dec{lvl}b.b"]), 0.0))
        c[f"dec{lvl}b"] = h
    hw = W["head.w"].reshape(-1)
    out = x_in + W["head.b"][0] + h @ hw
    return out, c


def backward(params, cache, g_out, rounding: bool = True, channels=CHANNELS):
    """Gradients of a scalar loss with dL/d(output) = g_out, through the
    stored (rounded) activations.  Every stored activation gradient is
    rounded like the activations; ReLU masks use the stored outputs
    (a > 0).  Returns {param name: gradient} (weight gradients unrounded)."""
    q = lambda a: _q(a, rounding)
    W = {k: (q(v) if k.endswith(".w") else np.asarray(v, dtype=np.float64)) for k, v in params.items()}
    nl = len(channels)
    g_out = np.asarray(g_out, dtype=np.float64)
    G = {}
    h = cache[f"dec0b"]
    G["head.w"] = (g_out[..., None] * h).sum(axis=(0, 1, 2, 3)).reshape(1, 1, -1)
    G["head.b"] = np.array([g_out.sum()])
    hw = W["head.w"].reshape(-1)
    dz = q(g_out[..., None] * hw * (h > 0))
    skip_grads = {}
    for lvl in range(0, nl - 1):
        # dz: gradient at dec{lvl}b's pre-activation.  Decoder level lvl is
        # dec{lvl}b <- dec{lvl}a <- concat(up{lvl}, enc{lvl}b), up{lvl} <- below
        a = cache[f"dec{lvl}a"]
        G[f"dec{lvl}b.w"], G[f"dec{lvl}b.b"] = conv3_wgrad(a, dz)
        dz = q(conv3_dgrad(dz, W[f"dec{lvl}b.w"]) * (a > 0))
        cat = np.concatenate([cache[f"up{lvl}"], cache[f"enc{lvl}b"]], axis=-1)
        G[f"dec{lvl}a.w"], G[f"dec{lvl}a.b"] = conv3_wgrad(cat, dz)
        dcat = q(conv3_dgrad(dz, W[f"dec{lvl}a.w"]))
        cu = channels[lvl]
        du, skip_grads[lvl] = dcat[..., :cu], dcat[..., cu:]
        below = cache[f"dec{lvl + 1}b"] if lvl + 1 < nl - 1 else cache[f"enc{nl - 1}b"]
        G[f"up{lvl}.w"], G[f"up{lvl}.b"] = up2_wgrad(below, du)
        dz = q(up2_dgrad(du, W[f"up{lvl}.w"]) * (below > 0))
    # dz: gradient at the bottleneck's enc{nl-1}b pre-activation
    for lvl in range(nl - 1, -1, -1):
        a = cache[f"enc{lvl}a"]
        G[f"enc{lvl}b.w"], G[f"enc{lvl}b.b"] = conv3_wgrad(a, dz)
        dz = q(conv3_dgrad(dz, W[f"enc{lvl}b.w"]) * (a > 0))
        inp = cache["x0"] if lvl == 0 else cache[f"pool{lvl}"]
        G[f"enc{lvl}a.w"], G[f"enc{lvl}a.b"] = conv3_wgrad(inp, dz)
        if lvl == 0:
            break
        dp = q(conv3_dgrad(dz, W[f"enc{lvl}a.w"]))
        e = cache[f"enc{lvl - 1}b"]
        dz = q((pool2_adjoint(dp) + skip_grads[lvl - 1]) * (e > 0))
    return G


def mse_loss(out, target) -> Tuple[float, np.ndarray]:
    """mean((out - target)^2) and its gradient 2 (out - target) / M."""
    d = np.asarray(out, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam(params, grads, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma & Ba, 2015) with bias correction, in place on FP64
    copies: m <- b1 m + (1 - b1) g; v <- b2 v + (1 - b2) g^2;
    w <- w - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k, g in grads.items():
        m = state.setdefault("m." + k, np.zeros_like(g))
        v = state.setdefault("v." + k, np.zeros_like(g))
        m *= beta1
        m += (1 - beta1) * g
        v *= beta2
        v += (1 - beta2) * g * g
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params
