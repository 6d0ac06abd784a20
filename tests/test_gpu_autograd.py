"""Differentiation through the projector (the paper's PyTorch operator
wrappers, section 2.8): A as a torch.autograd.Function whose backward is the
matched A^T kernel.

Checks: finite differences on 1000 voxels (exact for the quadratic
|Ax - y|^2 up to rounding), the dot-product identity through autograd,
torch.autograd.gradcheck on a tiny problem, and -- on the 512^3 x 720
workload -- the gradient of |Ax - y|^2 against the FP64 oracle on sampled
voxels.
"""
import numpy as np
import pytest

import synth
from synth import Geometry

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_10129_amd as P
    return P


def _f64_sq(t):
    return float((t.double() ** 2).sum())


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_finite_differences_on_1000_voxels(P, kind):
    """Central differences of f(x) = |Ax - y|^2 (FP64 sum of the FP32
    residual) against autograd's 2 A^T (Ax - y).  f is quadratic, so the
    central difference is exact for any step; eps = 0.1 max|x| keeps it
    above rounding."""
    geo = Geometry(DSD=1536.0, DSO=1000.0, nVoxel=(40, 48, 48), dVoxel=(1.0, 1.0, 1.0), nDetector=(48, 64),
                   dDetector=(1.6, 1.6))
    ang = synth.circular_angles(40)
    A = P.Projector(geo, ang, kind=kind)
    x0 = torch.from_numpy(synth.uniform_volume(geo, 61)).cuda()
    y = torch.from_numpy(synth.uniform_projections(geo, len(ang), 62)).cuda() * 20.0
    x = x0.clone().requires_grad_(True)
    loss = ((A(x) - y) ** 2).sum()
    loss.backward()
    g = x.grad.double().cpu().numpy().ravel()
    rng = np.random.Generator(np.random.PCG64(63))
    # 1000 voxels inside the FOV cylinder
    nz, ny, nx = geo.nVoxel
    sel = []
    while len(sel) < 1000:
        iz, iy, ix = rng.integers(nz), rng.integers(ny), rng.integers(nx)
        if (iy + 0.5 - ny / 2) ** 2 + (ix + 0.5 - nx / 2) ** 2 < (0.45 * nx) ** 2:
            sel.append((iz * ny + iy) * nx + ix)
    eps = 0.1 * float(x0.abs().max())
    fd = np.empty(len(sel))
    with torch.no_grad():
        flat = x0.clone().view(-1)
        for n, j in enumerate(sel):
            v = float(flat[j])
            flat[j] = v + eps
            fp = _f64_sq(A(flat.view(geo.nVoxel)) - y)
            flat[j] = v - eps
            fm = _f64_sq(A(flat.view(geo.nVoxel)) - y)
            flat[j] = v
            fd[n] = (fp - fm) / (2 * eps)
    gs = g[sel]
    err = np.abs(fd - gs) / np.maximum(np.abs(gs), 1e-2 * np.abs(gs).max())
    assert np.max(err) < 1e-3, np.max(err)


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_autograd_dot_product_and_batching(P, kind):
    """<A x, y> = <x, A^T y> on a batch of two, through the autograd
    operators; A.T's backward is A."""
    geo = Geometry(DSD=400.0, DSO=250.0, nVoxel=(20, 24, 28), dVoxel=(1.0, 1.0, 1.0), nDetector=(30, 40),
                   dDetector=(1.3, 1.3))
    ang = synth.circular_angles(16)
    A = P.Projector(geo, ang, kind=kind)
    g = torch.Generator(device="cuda").manual_seed(64)
    x = torch.rand((2,) + geo.nVoxel, generator=g, device="cuda")
    y = torch.rand((2, 16) + geo.nDetector, generator=g, device="cuda")
    ax = A(x)
    aty = A.T(y)
    assert ax.shape == (2, 16) + geo.nDetector and aty.shape == (2,) + geo.nVoxel
    for b in range(2):
        lhs = float((ax[b].double() * y[b].double()).sum())
        rhs = float((x[b].double() * aty[b].double()).sum())
        assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
    yv = y.clone().requires_grad_(True)
    (A.T(yv) * x).sum().backward()
    assert torch.allclose(yv.grad, A(x), rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_gradcheck_tiny(P, kind):
    geo = Geometry(DSD=60.0, DSO=40.0, nVoxel=(4, 4, 4), dVoxel=(1.0, 1.0, 1.0), nDetector=(4, 5),
                   dDetector=(1.4, 1.4), offDetector=(0.2, -0.3))
    ang = np.array([0.3, 1.9])
    A = P.Projector(geo, ang, kind=kind)
    x = torch.rand(geo.nVoxel, device="cuda", dtype=torch.float32, generator=torch.Generator(device="cuda").manual_seed(65))
    x.requires_grad_(True)
    assert torch.autograd.gradcheck(lambda t: A(t), (x,), eps=1e-2, atol=2e-3, rtol=2e-3)


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_gradient_vs_oracle_at_512(P, orc, kind):
    """512^3 x 720 views, 1024 x 768 detector: the autograd gradient of
    |Ax - y|^2 on 48 sampled FOV voxels (16 of them on the adjoint's brick
    faces) against the oracle's entry-by-entry FP64 gradient."""
    geo, ang = synth.workload("cbct512")
    xh = synth.uniform_volume(geo, 66)
    yh = synth.uniform_projections(geo, len(ang), 67) * 200.0
    A = P.Projector(geo, ang, kind=kind)
    x = torch.from_numpy(xh).cuda().requires_grad_(True)
    y = torch.from_numpy(yh).cuda()
    loss = ((A(x) - y) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(68))
    nz, ny, nx = geo.nVoxel
    iz = rng.integers(8, nz - 8, 32)
    iy = rng.integers(96, ny - 96, 32)
    ix = rng.integers(96, nx - 96, 32)
    # voxels on 16x16x8 brick faces (x or y = 0 or 15 mod 16, z = 0 or 7 mod 8)
    fz = rng.integers(1, nz // 8 - 1, 16) * 8 + rng.choice([0, 7], 16)
    fy = rng.integers(6, ny // 16 - 6, 16) * 16 + rng.choice([0, 15], 16)
    fx = rng.integers(6, nx // 16 - 6, 16) * 16 + rng.choice([0, 15], 16)
    iz, iy, ix = np.concatenate([iz, fz]), np.concatenate([iy, fy]), np.concatenate([ix, fx])
    got = x.grad[torch.from_numpy(iz).cuda(), torch.from_numpy(iy).cuda(), torch.from_numpy(ix).cuda()]
    got = got.double().cpu().numpy()
    want = orc.gradient_voxels(geo, ang, xh, yh, iz, iy, ix, kind)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert rel < 1e-4, rel
