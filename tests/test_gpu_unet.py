"""Parity of the BF16 U-Net kernels (the learned prior) with the FP64
oracle.  Inputs and weights are BF16-exact values from the shared
generators; outputs that the kernels round to BF16 are compared with the
oracle's FP64 result rounded the same way (at most a neighbouring BF16
value apart where FP32 and FP64 sums straddle a rounding boundary), sums
kept in FP32 against FP64 with a relative bound.  Sizes are ragged against
the kernels' 2 x 8 x 16 tiles; the full network runs at 16 x 24 x 32."""
import ctypes
import math

import numpy as np
import pytest

import synth
from oracle import unet as U

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_10129_amd as P
    return P


def _lib():
    from paper_2412_10129_amd import _lib as L
    return L


def _p(t, off=0):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr() + off * t.element_size())


def _s():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _bf(a):
    """numpy FP32 (BF16-exact) -> device bfloat16 tensor."""
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda().to(torch.bfloat16)


def _np(t):
    return t.float().cpu().numpy().astype(np.float64)


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(np.asarray(b).ravel()), 1e-300))


def _bf16_close(got, want_exact):
    """got: BF16 kernel output; want_exact: FP64 value before rounding."""
    want = U.bf16(want_exact)
    ulp = np.ldexp(1.0, np.frexp(np.abs(want_exact))[1] - 8)
    bad = np.abs(got - want) > 1.01 * ulp + 1e-30
    assert bad.mean() < 1e-3, bad.mean()
    assert _rel(got, want) < 2e-3


def _ws(nbytes):
    return torch.empty((nbytes + 15) // 4 + 4, dtype=torch.float32, device="cuda")


CONV_CASES = [
    # (n, d, h, w, c0, c1, cout)
    (1, 3, 5, 7, 16, 0, 16),
    (2, 5, 11, 19, 16, 16, 32),
    (1, 4, 9, 33, 32, 0, 64),
    (1, 2, 8, 16, 64, 64, 128),
    (1, 3, 6, 17, 128, 0, 16),
]


@pytest.mark.parametrize("case", CONV_CASES)
def test_conv3_forward(P, case):
    n, d, h, w, c0, c1, cout = case
    cin = c0 + c1
    x0 = synth.bf16_values((n, d, h, w, c0), 1)
    x1 = synth.bf16_values((n, d, h, w, c1), 2) if c1 else None
    wt = synth.bf16_values((cout, 27, cin), 3, -0.2, 0.2)
    b = synth.bf16_values((cout,), 4, -0.5, 0.5)
    out = torch.empty((n, d, h, w, cout), dtype=torch.bfloat16, device="cuda")
    tx0, tx1 = _bf(x0), (_bf(x1) if c1 else None)
    tw, tb = _bf(wt), torch.from_numpy(b).cuda()
    L = _lib()
    L.check(L.lib().ctmi_conv3d_bf16_fwd(n, d, h, w, _p(tx0), c0, c0, _p(tx1), c1, c1 if c1 else 8, _p(tw), _p(tb),
                                         cout, 1, _p(out), cout, _s()))
    xin = np.concatenate([x0, x1], -1) if c1 else x0
    want = np.maximum(U.conv3(xin, wt, b), 0.0)
    _bf16_close(_np(out), want)


@pytest.mark.parametrize("case", [(1, 3, 5, 7, 16, 32), (2, 4, 9, 18, 64, 32), (1, 2, 8, 17, 128, 128)])
def test_conv3_dgrad_with_mask_and_pack(P, case):
    n, d, h, w, cout, cin = case
    dz = synth.bf16_values((n, d, h, w, cout), 5)
    wm = np.random.Generator(np.random.PCG64(6)).standard_normal((cout, 27, cin)).astype(np.float32) * 0.1
    mask = synth.bf16_values((n, d, h, w, cin), 7)
    L = _lib()
    twm = torch.from_numpy(wm).cuda()
    wf = torch.empty((cout, 27, cin), dtype=torch.bfloat16, device="cuda")
    wd = torch.empty((cin, 27, cout), dtype=torch.bfloat16, device="cuda")
    L.check(L.lib().ctmi_conv3d_pack_weights(_p(twm), cout, cin, _p(wf), _p(wd), _s()))
    assert np.array_equal(_np(wf), U.bf16(wm))
    tdz, tm = _bf(dz), _bf(mask)
    dx = torch.empty((n, d, h, w, cin), dtype=torch.bfloat16, device="cuda")
    L.check(L.lib().ctmi_conv3d_bf16_dgrad(n, d, h, w, _p(tdz), cout, cout, _p(wd), cin, _p(tm), cin, _p(dx), cin,
                                           _s()))
    want = U.conv3_dgrad(dz, U.bf16(wm)) * (mask > 0)
    _bf16_close(_np(dx), want)


@pytest.mark.parametrize("case", [(1, 3, 5, 7, 16, 0, 16), (2, 5, 11, 19, 16, 16, 32), (1, 6, 9, 20, 64, 64, 128),
                                  (1, 4, 8, 16, 128, 0, 64)])
def test_conv3_wgrad(P, case):
    n, d, h, w, c0, c1, cout = case
    x0 = synth.bf16_values((n, d, h, w, c0), 8)
    x1 = synth.bf16_values((n, d, h, w, c1), 9) if c1 else None
    dz = synth.bf16_values((n, d, h, w, cout), 10)
    L = _lib()
    cin = c0 + c1
    ws = _ws(L.lib().ctmi_conv3d_wgrad_workspace_bytes(n, d, h, w, cin, cout))
    dw = torch.full((cout, 27, cin), 7.0, device="cuda")
    db = torch.full((cout,), 7.0, device="cuda")
    tx0, tx1, tdz = _bf(x0), (_bf(x1) if c1 else None), _bf(dz)
    for acc in (0, 1):
        L.check(L.lib().ctmi_conv3d_bf16_wgrad(n, d, h, w, _p(tx0), c0, c0, _p(tx1), c1, c1 if c1 else 8, _p(tdz),
                                               cout, cout, _p(dw), _p(db), acc, _p(ws), ws.numel() * 4, _s()))
    xin = np.concatenate([x0, x1], -1) if c1 else x0
    wdw, wdb = U.conv3_wgrad(xin, dz)
    assert _rel(dw.cpu().numpy() / 2, wdw) < 1e-5
    assert _rel(db.cpu().numpy() / 2, wdb) < 1e-5


def test_pool_up_skip_head_kernels(P):
    L = _lib()
    lib = L.lib()
    n, d, h, w = 2, 3, 5, 6          # coarse sizes
    c, cout = 32, 16
    fine = synth.bf16_values((n, 2 * d, 2 * h, 2 * w, c), 11)
    tf = _bf(fine)
    pooled = torch.empty((n, d, h, w, c), dtype=torch.bfloat16, device="cuda")
    L.check(lib.ctmi_pool2(n, d, h, w, c, _p(tf), c, _p(pooled), c, _s()))
    _bf16_close(_np(pooled), U.pool2(fine))
    # transposed convolution, its data gradient (with mask) and weight gradient
    x = synth.bf16_values((n, d, h, w, c), 12)
    wt = synth.bf16_values((cout, 8, c), 13, -0.3, 0.3)
    b = synth.bf16_values((cout,), 14)
    tx, tw, tb = _bf(x), _bf(wt), torch.from_numpy(b).cuda()
    up = torch.empty((n, 2 * d, 2 * h, 2 * w, cout), dtype=torch.bfloat16, device="cuda")
    L.check(lib.ctmi_upsample2(n, d, h, w, _p(tx), c, c, _p(tw), _p(tb), cout, _p(up), cout, _s()))
    _bf16_close(_np(up), U.up2(x, wt, b))
    # the gradient arrives as the first half of a concatenation gradient
    gcat = synth.bf16_values((n, 2 * d, 2 * h, 2 * w, 2 * cout), 15)
    tg = _bf(gcat)
    below = synth.bf16_values((n, d, h, w, c), 16)
    tbel = _bf(below)
    dx = torch.empty((n, d, h, w, c), dtype=torch.bfloat16, device="cuda")
    L.check(lib.ctmi_upsample2_dgrad(n, d, h, w, _p(tg), cout, 2 * cout, _p(tw), c, _p(tbel), c, _p(dx), c, _s()))
    _bf16_close(_np(dx), U.up2_dgrad(gcat[..., :cout], wt) * (below > 0))
    ws = _ws(lib.ctmi_upsample2_wgrad_workspace_bytes(n, d, h, w, c, cout))
    dw = torch.empty((cout, 8, c), device="cuda")
    db = torch.empty((cout,), device="cuda")
    L.check(lib.ctmi_upsample2_wgrad(n, d, h, w, _p(tx), c, c, _p(tg), cout, 2 * cout, _p(dw), _p(db), 0, _p(ws),
                                     ws.numel() * 4, _s()))
    wdw, wdb = U.up2_wgrad(x, gcat[..., :cout])
    assert _rel(dw.cpu().numpy(), wdw) < 1e-5 and _rel(db.cpu().numpy(), wdb) < 1e-5
    # skip gradient: mask(e) * (dp[parent] / 8 + second half of dcat)
    e = synth.bf16_values((n, 2 * d, 2 * h, 2 * w, cout), 17)
    dp = synth.bf16_values((n, d, h, w, cout), 18)
    te, tdp = _bf(e), _bf(dp)
    dze = torch.empty((n, 2 * d, 2 * h, 2 * w, cout), dtype=torch.bfloat16, device="cuda")
    L.check(lib.ctmi_pool2_skip_grad(n, 2 * d, 2 * h, 2 * w, cout, _p(te), cout, _p(tdp), cout, _p(tg, cout),
                                     2 * cout, _p(dze), cout, _s()))
    _bf16_close(_np(dze), (U.pool2_adjoint(dp) + gcat[..., cout:]) * (e > 0))


@pytest.mark.parametrize("cin,cout,mask", [(32, 16, True), (64, 32, False), (128, 64, True)])
def test_up2_gradients_every_level(P, cin, cout, mask):
    """The up-convolution's data gradient (with and without the ReLU mask of
    its input) and weight gradient at each level's channel counts (the MFMA
    kernels' tile counts), on a ragged coarse grid (the last wave and the
    last voxel chunk partly empty), against the oracle's adjoints of the
    transposed convolution."""
    L = _lib()
    lib = L.lib()
    n, d, h, w = 1, 3, 5, 7
    wt = synth.bf16_values((cout, 8, cin), 301 + cin, -0.3, 0.3)
    gr = synth.bf16_values((n, 2 * d, 2 * h, 2 * w, cout + 8), 302 + cin)
    below = synth.bf16_values((n, d, h, w, cin), 303 + cin)
    tw, tg, tbel = _bf(wt), _bf(gr), _bf(below)
    dx = torch.empty((n, d, h, w, cin), dtype=torch.bfloat16, device="cuda")
    L.check(lib.ctmi_upsample2_dgrad(n, d, h, w, _p(tg), cout, cout + 8, _p(tw), cin, _p(tbel) if mask else None,
                                     cin, _p(dx), cin, _s()))
    want = U.up2_dgrad(gr[..., :cout], wt)
    if mask:
        want = want * (below > 0)
    _bf16_close(_np(dx), want)
    x = synth.bf16_values((n, d, h, w, cin + 16), 304 + cin)
    tx = _bf(x)
    ws = _ws(lib.ctmi_upsample2_wgrad_workspace_bytes(n, d, h, w, cin, cout))
    dw = torch.empty((cout, 8, cin), device="cuda")
    L.check(lib.ctmi_upsample2_wgrad(n, d, h, w, _p(tx), cin, cin + 16, _p(tg), cout, cout + 8, _p(dw), None, 0,
                                     _p(ws), ws.numel() * 4, _s()))
    wdw, _ = U.up2_wgrad(x[..., :cin], gr[..., :cout])
    assert _rel(dw.cpu().numpy(), wdw) < 1e-5, _rel(dw.cpu().numpy(), wdw)


def test_head_loss_and_adam(P):
    L = _lib()
    lib = L.lib()
    nv = 3000
    xin = np.random.Generator(np.random.PCG64(19)).random(nv).astype(np.float32)
    act = synth.bf16_values((nv, 16), 20)
    hw = synth.bf16_values((16,), 21, -0.5, 0.5)
    hb = np.array([0.25], dtype=np.float32)
    tgt = np.random.Generator(np.random.PCG64(22)).random(nv).astype(np.float32)
    txin, tact, thw, thb = torch.from_numpy(xin).cuda(), _bf(act), _bf(hw), torch.from_numpy(hb).cuda()
    out = torch.empty(nv, device="cuda")
    L.check(lib.ctmi_unet_head(nv, _p(txin), _p(tact), 16, 16, _p(thw), _p(thb), _p(out), _s()))
    want = xin + hb[0] + act.astype(np.float64) @ hw
    assert np.max(np.abs(out.cpu().numpy() - want)) < 1e-5
    ws = torch.empty(lib.ctmi_unet_head_workspace_bytes() // 8 + 2, dtype=torch.float64, device="cuda")
    sums = torch.empty(18, dtype=torch.float64, device="cuda")
    dhead = torch.empty(17, device="cuda")
    dz = torch.empty((nv, 16), dtype=torch.bfloat16, device="cuda")
    ttgt = torch.from_numpy(tgt).cuda()
    L.check(lib.ctmi_unet_head_mse_bwd(nv, _p(out), _p(ttgt), _p(tact), 16, _p(thw), _p(dz), 16, _p(sums),
                                       _p(dhead), _p(ws), ws.numel() * 8, _s()))
    o = out.double().cpu().numpy()
    loss, g = U.mse_loss(o, tgt)
    s = sums.cpu().numpy()
    assert abs(s[17] / nv - loss) < 1e-6 * loss
    assert _rel(s[:16], g @ act) < 1e-5 and abs(s[16] - g.sum()) < 1e-5 * np.abs(g).sum()
    assert _rel(dhead.cpu().numpy(), s[:17]) < 1e-6
    _bf16_close(_np(dz), g[:, None] * hw[None, :] * (act > 0))
    # Adam: three steps against the oracle's FP64 Adam
    rng = np.random.Generator(np.random.PCG64(23))
    w0 = rng.standard_normal(1000).astype(np.float32)
    tw = torch.from_numpy(w0.copy()).cuda()
    tm, tv = torch.zeros_like(tw), torch.zeros_like(tw)
    pw, st = {"w": w0.astype(np.float64)}, {}
    for t in range(1, 4):
        g = rng.standard_normal(1000).astype(np.float32)
        L.check(lib.ctmi_adam_step(_p(tw), _p(tm), _p(tv), _p(torch.from_numpy(g).cuda()), 1000, 1e-3, 0.9, 0.999,
                                   1e-8, t, _s()))
        U.adam(pw, {"w": g.astype(np.float64)}, st)
    assert np.max(np.abs(tw.cpu().numpy() - pw["w"])) < 1e-6


def _load_oracle_params(net, channels):
    """Master weights of the device net as oracle FP64 dicts (the first
    convolution unpadded)."""
    p = {}
    for name, kind, shp in U.layer_shapes(channels):
        w = net.w(name).cpu().numpy().astype(np.float64)
        p[name + ".w"] = w[..., :shp[2]]
        p[name + ".b"] = net.b(name).cpu().numpy().astype(np.float64)
    return p


def _net_and_batch(P):
    net = P.UNet(seed=3)
    # small nonzero biases so every ReLU path is exercised (seeded host values)
    for i, (name, _, _) in enumerate(net.layers):
        bias = synth.bf16_values(tuple(net.b(name).shape), 240 + i, -0.05, 0.05)
        net.b(name).copy_(torch.from_numpy(bias))
    net.pack()
    x = synth.bf16_values((1, 16, 24, 32), 25, 0.0, 1.0)
    tgt = (x * 0.8 + 0.1).astype(np.float32)
    return net, x, tgt


def test_unet_end_to_end_vs_oracle(P):
    """The whole network against the oracle run on the same inputs.  BF16
    rounding boundaries amplify the FP32-vs-FP64 difference of the sums: in
    the oracle itself a 1e-7 relative perturbation of every convolution
    output moves the network's contribution by 4e-3 and the deepest weight
    gradients by up to 9e-2 (mean 1.7e-2) at this size, so the bars here are
    a few times those; the single-kernel tests above pin every stage on
    independent seeded inputs."""
    net, x, tgt = _net_and_batch(P)
    tx, tt = torch.from_numpy(x).cuda(), torch.from_numpy(tgt).cuda()
    out, cache = net.forward(tx, keep=True)
    sq = net.backward(cache, tt, out)
    torch.cuda.synchronize()
    params = _load_oracle_params(net, U.CHANNELS)
    o_out, o_cache = U.forward(params, x.astype(np.float64))
    loss, gr = U.mse_loss(o_out, tgt)
    G = U.backward(params, o_cache, gr)
    got = out.cpu().numpy().astype(np.float64)
    assert _rel(got - x, o_out - x) < 1.5e-2
    assert abs(float(sq.cpu()) / x.size - loss) < 2e-3 * loss
    # the padded input channels of the first convolution get exactly zero gradient
    assert not np.any(net.w("enc0a", grad=True).cpu().numpy()[..., 1:])
    worst = {}
    for name, kind, shp in U.layer_shapes():
        gw = net.w(name, grad=True).cpu().numpy().astype(np.float64)[..., :shp[2]]
        gb = net.b(name, grad=True).cpu().numpy().astype(np.float64)
        worst[name] = max(_rel(gw, G[name + ".w"]), _rel(gb, G[name + ".b"]) if np.any(G[name + ".b"]) else 0.0)
    assert max(worst.values()) < 0.3, worst
    assert np.mean(list(worst.values())) < 0.06, worst


def test_unet_training_reduces_loss(P):
    net = P.UNet(seed=4)
    rng = np.random.Generator(np.random.PCG64(26))
    clean = np.zeros((2, 16, 16, 16), dtype=np.float32)
    clean[:, 4:12, 4:12, 4:12] = 1.0
    noisy = (clean + rng.standard_normal(clean.shape).astype(np.float32) * 0.1).astype(np.float32)
    tx, tt = torch.from_numpy(noisy).cuda(), torch.from_numpy(clean).cuda()
    first = None
    for it in range(60):
        sq = float(net.train_step(tx, tt).cpu())
        if first is None:
            first = sq
    final = float(((net.forward(tx) - tt) ** 2).sum().cpu())
    assert final < 0.5 * first, (first, final)


def test_pnp_cgls_vs_oracle(P, orc):
    """PnP-CGLS with the (untrained) U-Net on the GPU against the oracle's
    PnP-CGLS with the oracle network carrying the same weights.  The
    acceptance ratio is chosen away from every proposal's residual ratio so
    that both sides take the same decisions."""
    from synth import Geometry
    geo = Geometry(DSD=400.0, DSO=250.0, nVoxel=(32, 32, 32), dVoxel=(1.0, 1.0, 1.0), nDetector=(48, 48),
                   dDetector=(1.3, 1.3))
    ang = synth.circular_angles(16)
    x_gt = synth.textured_phantom(geo, 7)
    net = P.UNet(seed=5)
    params = _load_oracle_params(net, U.CHANNELS)
    den = lambda x: U.forward(params, np.asarray(x, dtype=np.float64)[None])[0][0]
    b = orc.forward(geo, ang, x_gt.astype(np.float64), "interp").astype(np.float32)
    chosen = None
    for ratio in (1.05, 1.5, 0.9, 3.0, 0.5):
        xo, ho = orc.pnp_cgls(geo, ang, b.astype(np.float64), 10, den, every=5, ratio=ratio, kind="interp")
        if all(abs(math.log(q / ratio)) > 0.02 for q in ho["ratios"]):
            chosen = ratio
            break
    assert chosen is not None, ho["ratios"]
    plan = P.Plan(geo, ang)
    xg, hg = P.pnp_cgls(plan, torch.from_numpy(b).cuda(), 10, net, every=5, ratio=chosen, kind="interp")
    assert hg["accepted"] == ho["accepted"], (hg["ratios"], ho["ratios"])
    assert np.allclose(hg["ratios"], ho["ratios"], rtol=2e-3)
    assert _rel(xg.cpu().numpy().astype(np.float64), xo) < 1e-3
    assert np.allclose(hg["resid"], ho["resid"], rtol=1e-3)
