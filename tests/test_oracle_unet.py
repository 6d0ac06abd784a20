"""Pins of the U-Net oracle (the learned prior used plug-and-play in CGLS)
against things other than itself: torch's own FP64 conv3d / conv_transpose3d
/ avg_pool3d and autograd on the CPU (library routines), pure-Python loops
on tiny inputs, adjoint identities, torch's BF16 conversion, and
torch.optim.Adam."""
import itertools
import math

import numpy as np
import pytest

import synth
from oracle import unet as U

torch = pytest.importorskip("torch")
F = torch.nn.functional


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))


def _ncdhw(x):          # [N, D, H, W, C] -> [N, C, D, H, W]
    return _t(x).permute(0, 4, 1, 2, 3)


def _ndhwc(x):
    return x.permute(0, 2, 3, 4, 1).detach().numpy()


def _w3(w):             # [Cout, 27, Cin] -> torch [Cout, Cin, 3, 3, 3]
    co, _, ci = w.shape
    return _t(np.asarray(w).reshape(co, 3, 3, 3, ci).transpose(0, 4, 1, 2, 3))


def _w2(w):             # [Cout, 8, Cin] -> torch transposed [Cin, Cout, 2, 2, 2]
    co, _, ci = w.shape
    return _t(np.asarray(w).reshape(co, 2, 2, 2, ci).transpose(4, 0, 1, 2, 3))


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ------------------------------------------------------------- rounding
def test_bf16_rounding_matches_torch_and_hand_cases():
    rng = _rng(1)
    a = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        np.array([0.0, -0.0, 1.0, -2.5])])
    want = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).double().numpy()
    assert np.array_equal(U.bf16(a.astype(np.float32)), want)
    # ties go to the even neighbour: ulp(1) = 2^-7 in BF16
    assert U.bf16(1.0 + 2.0 ** -8) == 1.0
    assert U.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert U.bf16(-(1.0 + 2.0 ** -8 + 2.0 ** -20)) == -(1.0 + 2.0 ** -7)
    assert U.bf16(3.0) == 3.0 and U.bf16(1.0 / 3.0) == 0.333984375


def test_bf16_values_generator_is_exact():
    a = synth.bf16_values((1000,), 2)
    assert np.array_equal(U.bf16(a), a.astype(np.float64))


# ---------------------------------------------------------- convolution
def test_conv3_brute_force_tiny():
    rng = _rng(3)
    x = rng.standard_normal((1, 3, 2, 4, 2))
    w = rng.standard_normal((3, 27, 2))
    b = rng.standard_normal(3)
    got = U.conv3(x, w, b)
    _, D, H, W, C = x.shape
    for z, y, xx, co in itertools.product(range(D), range(H), range(W), range(3)):
        s = b[co]
        for kz, ky, kx in itertools.product(range(3), range(3), range(3)):
            zz, yy, xi = z + kz - 1, y + ky - 1, xx + kx - 1
            if 0 <= zz < D and 0 <= yy < H and 0 <= xi < W:
                for ci in range(C):
                    s += x[0, zz, yy, xi, ci] * w[co, 9 * kz + 3 * ky + kx, ci]
        assert abs(got[0, z, y, xx, co] - s) < 1e-12


def test_conv3_matches_torch_conv3d():
    rng = _rng(4)
    x = rng.standard_normal((2, 5, 6, 7, 4))
    w = rng.standard_normal((6, 27, 4))
    b = rng.standard_normal(6)
    want = _ndhwc(F.conv3d(_ncdhw(x), _w3(w), _t(b), padding=1))
    assert np.max(np.abs(U.conv3(x, w, b) - want)) < 1e-12


def test_conv3_adjoints():
    rng = _rng(5)
    x = rng.standard_normal((2, 5, 4, 6, 3))
    w = rng.standard_normal((5, 27, 3))
    g = rng.standard_normal((2, 5, 4, 6, 5))
    lhs = np.vdot(U.conv3(x, w), g)
    assert abs(lhs - np.vdot(x, U.conv3_dgrad(g, w))) < 1e-10 * abs(lhs)
    dw, db = U.conv3_wgrad(x, g)
    assert abs(lhs - np.vdot(w, dw)) < 1e-10 * abs(lhs)
    assert np.allclose(db, g.sum(axis=(0, 1, 2, 3)), rtol=1e-13)


def test_up2_and_pool2_match_torch_and_adjoints():
    rng = _rng(6)
    x = rng.standard_normal((2, 3, 2, 4, 5))
    w = rng.standard_normal((4, 8, 5))
    b = rng.standard_normal(4)
    want = _ndhwc(F.conv_transpose3d(_ncdhw(x), _w2(w), _t(b), stride=2))
    assert np.max(np.abs(U.up2(x, w, b) - want)) < 1e-12
    g = rng.standard_normal((2, 6, 4, 8, 4))
    lhs = np.vdot(U.up2(x, w), g)
    assert abs(lhs - np.vdot(x, U.up2_dgrad(g, w))) < 1e-10 * abs(lhs)
    dw, db = U.up2_wgrad(x, g)
    assert abs(lhs - np.vdot(w, dw)) < 1e-10 * abs(lhs)
    y = rng.standard_normal((2, 6, 4, 8, 3))
    want = _ndhwc(F.avg_pool3d(_ncdhw(y), 2))
    assert np.max(np.abs(U.pool2(y) - want)) < 1e-13
    gp = rng.standard_normal((2, 3, 2, 4, 3))
    assert abs(np.vdot(U.pool2(y), gp) - np.vdot(y, U.pool2_adjoint(gp))) < 1e-10


# --------------------------------------------------------------- network
CH = (4, 8, 8, 8)


def _torch_unet(params, x_in, rounding, channels=CH):
    """The same network written with torch's own layers.  With rounding,
    stored values go through BF16 (straight-through in the backward) and
    gradient hooks round the gradients the oracle stores."""
    P = {k: _t(v).requires_grad_(True) for k, v in params.items()}
    q = (lambda a: a + (a.to(torch.float32).to(torch.bfloat16).double() - a).detach()) if rounding else (lambda a: a)

    def hook(t):
        if rounding:
            t.register_hook(lambda g: g.to(torch.float32).to(torch.bfloat16).double())
        return t

    Wq = {k: (q(v) if k.endswith(".w") else v) for k, v in P.items()}
    conv = lambda h, n: hook(F.conv3d(h, _w3_t(Wq[n + ".w"]), Wq[n + ".b"], padding=1))
    xt = _t(x_in)[:, None]
    h = q(xt)
    skips = []
    nl = len(channels)
    for lvl in range(nl):
        h = q(F.relu(conv(h, f"enc{lvl}a")))
        h = q(F.relu(conv(h, f"enc{lvl}b")))
        if lvl < nl - 1:
            skips.append(h)
            h = hook(q(F.avg_pool3d(h, 2)))
    for lvl in range(nl - 2, -1, -1):
        u = q(F.conv_transpose3d(h, _w2_t(Wq[f"up{lvl}.w"]), Wq[f"up{lvl}.b"], stride=2))
        cat = hook(torch.cat([u, skips[lvl]], dim=1))
        h = q(F.relu(conv(cat, f"dec{lvl}a")))
        h = q(F.relu(conv(h, f"dec{lvl}b")))
    head = torch.einsum("ncdhw,c->ndhw", h, Wq["head.w"].reshape(-1)) + Wq["head.b"][0]
    return xt[:, 0] + head, P


def _w3_t(w):
    co, _, ci = w.shape
    return w.reshape(co, 3, 3, 3, ci).permute(0, 4, 1, 2, 3)


def _w2_t(w):
    co, _, ci = w.shape
    return w.reshape(co, 2, 2, 2, ci).permute(4, 0, 1, 2, 3)


@pytest.mark.parametrize("rounding", [False, True])
def test_unet_forward_backward_matches_torch_autograd(rounding):
    params = U.init_params(7, CH)
    rng = _rng(10)
    for k in sorted(params):
        if k.endswith(".b"):
            params[k] = rng.standard_normal(params[k].shape) * 0.05
    x = synth.bf16_values((2, 16, 16, 8), 8, 0.0, 1.0).astype(np.float64)
    target = x * 0.9 + 0.05
    out, cache = U.forward(params, x, rounding=rounding, channels=CH)
    loss, g = U.mse_loss(out, target)
    G = U.backward(params, cache, g, rounding=rounding, channels=CH)
    tout, P = _torch_unet(params, x, rounding)
    tl = ((tout - _t(target)) ** 2).mean()
    tl.backward()
    assert np.max(np.abs(out - tout.detach().numpy())) < 1e-10
    assert abs(loss - float(tl.detach())) < 1e-12
    for k in params:
        want = P[k].grad.numpy()
        got = G[k]
        err = np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300)
        # rounding: a gradient computed in a different order may round to
        # the neighbouring BF16 value at a few points
        assert err < (1e-10 if not rounding else 1e-3), (k, err)


def test_param_count_and_layers():
    assert U.param_count() == 1400561
    names = [n for n, _, _ in U.layer_shapes()]
    assert names[:2] == ["enc0a", "enc0b"] and names[-1] == "head" and len(names) == 18


def test_adam_matches_torch_optim():
    rng = _rng(9)
    p = {"a": rng.standard_normal((3, 4)), "b": rng.standard_normal(5)}
    tp = {k: _t(v.copy()).requires_grad_(True) for k, v in p.items()}
    opt = torch.optim.Adam(list(tp.values()), lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    state = {}
    for step in range(4):
        g = {k: rng.standard_normal(v.shape) for k, v in p.items()}
        for k in tp:
            tp[k].grad = _t(g[k])
        opt.step()
        U.adam(p, g, state)
    for k in p:
        assert np.max(np.abs(p[k] - tp[k].detach().numpy())) < 1e-14
