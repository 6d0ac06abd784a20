"""Checkpoint and resume: a CGLS run, an OS-SART run and a U-Net training run
stopped part way, written with torch.save, read back with the safe loader
into fresh objects and continued, end bit for bit where the uninterrupted run
ends (every kernel on these paths sums in a fixed order, so a resumed run
repeats the same arithmetic)."""
import io

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_10129_amd as P
    return P


@pytest.fixture(scope="module")
def problem(P):
    geo, ang = synth.workload("head64")
    plan = P.Plan(geo, ang)
    x = torch.from_numpy(synth.voxelize(geo, synth.head_phantom(geo), dtype=np.float32)).cuda()
    b = plan.forward(x, kind="interp")
    return plan, b


def _roundtrip(P, state):
    f = io.BytesIO()
    P.save_state(state, f)
    f.seek(0)
    return P.load_state(f, device="cuda")


def test_cgls_resumes_bit_for_bit(P, problem):
    plan, b = problem
    x8, h8 = P.cgls(plan, b, 8, kind="interp")
    _, h4 = P.cgls(plan, b, 4, kind="interp")
    st = _roundtrip(P, h4["state"])
    assert st["k"] == 4
    seen = []
    x8r, h8r = P.cgls(plan, b, 4, kind="interp", state=st, snapshots=(6,), callback=lambda k, x: seen.append(k))
    assert seen == [5, 6, 7, 8]
    assert torch.equal(x8r, x8)
    assert np.array_equal(h8r["resid"], h8["resid"][4:])
    assert np.array_equal(h8r["gamma"], h8["gamma"][4:])
    assert h8r["state"]["k"] == 8 and torch.equal(h8r["state"]["p"], h8["state"]["p"])
    with pytest.raises(ValueError):
        P.cgls(plan, b, 1, kind="interp", state=st, x0=x8)


def test_os_sart_resumes_mid_pass_bit_for_bit(P, problem):
    plan, b = problem
    solver = P.OSSART(plan, 8, "interp")
    assert len(solver.blocks) == 8
    x = torch.zeros(plan.vol_shape, device="cuda")
    for _ in range(2):
        solver.sweep(x, b, 1.0, True)
    y = torch.zeros(plan.vol_shape, device="cuda")
    solver.sweep(y, b, 1.0, True)
    solver.sweep(y, b, 1.0, True, first=0, last=3)
    st = _roundtrip(P, P.OSSART.checkpoint(y, 1, 3))
    fresh = P.OSSART(plan, 8, "interp")
    z = st["x"].clone()
    fresh.sweep(z, b, 1.0, True, first=st["next_block"])
    assert st["passes"] + 1 == 2
    assert torch.equal(z, x)
    with pytest.raises(ValueError):
        fresh.sweep(z, b, 1.0, True, first=5, last=3)


def test_unet_training_resumes_bit_for_bit(P):
    from paper_2412_10129_amd import learned
    g = torch.Generator(device="cuda").manual_seed(11)
    inputs = [torch.rand((24, 24, 24), device="cuda", generator=g) for _ in range(2)]
    targets = [torch.rand((24, 24, 24), device="cuda", generator=g) for _ in range(2)]
    kw = dict(crop=16, batch=2, log_every=1000, log=lambda *a: None)
    a = P.UNet(seed=0)
    learned.train(a, inputs, targets, 4, rng=np.random.Generator(np.random.PCG64(5)), **kw)
    b = P.UNet(seed=0)
    rb = np.random.Generator(np.random.PCG64(5))
    learned.train(b, inputs, targets, 2, rng=rb, **kw)
    f = io.BytesIO()
    torch.save(learned.training_checkpoint(b, rb), f)
    f.seek(0)
    sd = torch.load(f, map_location="cpu", weights_only=True)
    c = P.UNet(seed=1)   # other initial weights: everything must come from the checkpoint
    rc = learned.restore_training(c, sd)
    assert c.t == 2
    learned.train(c, inputs, targets, 2, rng=rc, **kw)
    assert c.t == a.t == 4
    assert torch.equal(c.params, a.params)
    assert torch.equal(c.m, a.m) and torch.equal(c.v, a.v)
