"""Parity at full size, in the benchmark's launch configuration.

512^3 x 720 views (1024 x 768 detector): every operator is run on the whole
workload and sampled outputs are compared with the FP64 oracle computed
entry by entry (rays, voxels, filter rows).  1024^3 x 1440 views (1536^2
detector, 13.6 GB of projections, offsets beyond 2^31): closed forms (ray
chords through the volume box, the FDK backprojection of a constant),
linearity over view ranges, and the oracle on a view subset.
"""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_10129_amd as P
    return P


@pytest.fixture(scope="module")
def cbct(P):
    geo, ang = synth.workload("cbct512")
    xh = synth.uniform_volume(geo, 71)
    yh = synth.uniform_projections(geo, len(ang), 72)
    plan = P.Plan(geo, ang)
    x = torch.from_numpy(xh).cuda()
    y = torch.from_numpy(yh).cuda()
    return dict(geo=geo, ang=ang, xh=xh, yh=yh, y64=yh.astype(np.float64), plan=plan, x=x, y=y)


def _fov_voxels(geo, n, seed, rmax=0.9):
    rng = np.random.Generator(np.random.PCG64(seed))
    nz, ny, nx = geo.nVoxel
    out = []
    while len(out) < n:
        iz, iy, ix = int(rng.integers(nz)), int(rng.integers(ny)), int(rng.integers(nx))
        if (iy + 0.5 - ny / 2) ** 2 + (ix + 0.5 - nx / 2) ** 2 < (rmax * nx / 2) ** 2:
            out.append((iz, iy, ix))
    return [np.array(c) for c in zip(*out)]


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_512_forward_sampled_rays(P, orc, cbct, kind):
    geo, ang = cbct["geo"], cbct["ang"]
    out = cbct["plan"].forward(cbct["x"], kind=kind)
    rng = np.random.Generator(np.random.PCG64(73))
    n = 2048
    views = rng.integers(0, len(ang), n)
    ivs = rng.integers(0, geo.nDetector[0], n)
    ius = rng.integers(0, geo.nDetector[1], n)
    got = out[torch.from_numpy(views).cuda(), torch.from_numpy(ivs).cuda(), torch.from_numpy(ius).cuda()]
    got = got.double().cpu().numpy()
    want = orc.forward_rays(geo, ang, cbct["xh"], views, ivs, ius, kind)
    assert _rel(got, want) < 1e-4, _rel(got, want)


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_512_backward_sampled_voxels_and_determinism(P, orc, cbct, kind):
    geo, ang = cbct["geo"], cbct["ang"]
    out = cbct["plan"].backproject(cbct["y"], kind=kind)
    again = cbct["plan"].backproject(cbct["y"], kind=kind)
    assert torch.equal(out, again)          # fixed-point accumulation: bit-reproducible
    iz, iy, ix = _fov_voxels(geo, 24, 74)
    got = out[torch.from_numpy(iz).cuda(), torch.from_numpy(iy).cuda(), torch.from_numpy(ix).cuda()]
    got = got.double().cpu().numpy()
    want = orc.adjoint_voxels(geo, ang, cbct["y64"], iz, iy, ix, kind)
    assert _rel(got, want) < 1e-4, _rel(got, want)


def _brick_face_voxels(geo, n, seed):
    """Voxels on the adjoint's brick faces, edges and corners (16 x 16 x 8
    bricks: x or y = 0 or 15 mod 16, z = 0 or 7 mod 8), where its
    neighbour-shell additions land, inside the FOV cylinder."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nz, ny, nx = geo.nVoxel
    out = []
    while len(out) < n:
        bx, by, bz = int(rng.integers(nx // 16)), int(rng.integers(ny // 16)), int(rng.integers(nz // 8))
        kind = int(rng.integers(7))            # 1..7: faces (1 axis), edges (2), corners (3); bit per axis
        kind += 1
        lx = (0 if rng.integers(2) else 15) if kind & 1 else int(rng.integers(1, 15))
        ly = (0 if rng.integers(2) else 15) if kind & 2 else int(rng.integers(1, 15))
        lz = (0 if rng.integers(2) else 7) if kind & 4 else int(rng.integers(1, 7))
        iz, iy, ix = bz * 8 + lz, by * 16 + ly, bx * 16 + lx
        if (iy + 0.5 - ny / 2) ** 2 + (ix + 0.5 - nx / 2) ** 2 < (0.9 * nx / 2) ** 2:
            out.append((iz, iy, ix))
    return [np.array(c) for c in zip(*out)]


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_512_backward_brick_faces_and_interior(P, orc, cbct, kind):
    """A^T at 512 brick-face, edge and corner voxels and 256 random interior
    ones (rel-L2 1e-4 over each set, and every voxel within 1e-3)."""
    geo, ang = cbct["geo"], cbct["ang"]
    out = cbct["plan"].backproject(cbct["y"], kind=kind)
    for name, (iz, iy, ix) in (("faces", _brick_face_voxels(geo, 512, 81)), ("random", _fov_voxels(geo, 256, 82))):
        got = out[torch.from_numpy(iz).cuda(), torch.from_numpy(iy).cuda(), torch.from_numpy(ix).cuda()]
        got = got.double().cpu().numpy()
        want = orc.adjoint_voxels(geo, ang, cbct["y64"], iz, iy, ix, kind)
        assert _rel(got, want) < 1e-4, (name, _rel(got, want))
        assert np.max(np.abs(got / want - 1.0)) < 1e-3, name


def test_512_fdk_backprojector_sampled_voxels(P, orc, cbct):
    geo, ang = cbct["geo"], cbct["ang"]
    out = cbct["plan"].backproject(cbct["y"], kind="fdk")
    iz, iy, ix = _fov_voxels(geo, 64, 75, rmax=1.0)
    got = out[torch.from_numpy(iz).cuda(), torch.from_numpy(iy).cuda(), torch.from_numpy(ix).cuda()]
    want = orc.bfdk_voxels(geo, ang, cbct["y64"], iz, iy, ix)
    assert _rel(got.double().cpu().numpy(), want) < 1e-5


def test_512_fdk_filter_sampled_views(P, orc, cbct):
    geo, ang = cbct["geo"], cbct["ang"]
    out = cbct["plan"].fdk_filter(cbct["y"])
    for k in (0, 359, 719):
        want = orc.fdk_filter(geo, cbct["y64"][k:k + 1], ntotal=len(ang))
        assert _rel(out[k].cpu().numpy(), want) < 1e-5


# --------------------------------------------------------------- 1024^3
@pytest.fixture(scope="module")
def large(P):
    geo, ang = synth.workload("large1024")
    plan = P.Plan(geo, ang)
    return dict(geo=geo, ang=ang, plan=plan)


def _box_chords(geo, ang, views, ivs, ius, orc):
    nz, ny, nx = geo.nVoxel
    dz, dy, dx = geo.dVoxel
    oz, oy, ox = geo.offOrigin
    bl = np.array([ox - nx * dx / 2, oy - ny * dy / 2, oz - nz * dz / 2])
    bh = -bl + 2 * np.array([ox, oy, oz])
    out = np.zeros(len(views))
    for n, (k, iv, iu) in enumerate(zip(views, ivs, ius)):
        S, Pp = orc.ray_endpoints(geo, ang[k], float(iv), float(iu))
        d = Pp - S
        with np.errstate(divide="ignore"):
            a_lo, a_hi = (bl - S) / d, (bh - S) / d
        a0 = max(0.0, np.max(np.minimum(a_lo, a_hi)))
        a1 = min(1.0, np.min(np.maximum(a_lo, a_hi)))
        out[n] = max(a1 - a0, 0.0) * np.linalg.norm(d)
    return out


def test_1024_interp_forward_sampled_rays(P, orc, large):
    """The interpolated projector at 1024^3 x 1440 (offsets past 2^31 in the
    projections) on a U(0,1) volume, at 1024 rays against the oracle."""
    geo, ang, plan = large["geo"], large["ang"], large["plan"]
    xh = synth.uniform_volume(geo, 83)
    out = plan.forward(torch.from_numpy(xh).cuda(), kind="interp")
    rng = np.random.Generator(np.random.PCG64(84))
    n = 1024
    views = np.concatenate([rng.integers(0, len(ang), n - 64), np.full(64, len(ang) - 1)])
    ivs = rng.integers(0, geo.nDetector[0], n)
    ius = rng.integers(0, geo.nDetector[1], n)
    got = out[torch.from_numpy(views).cuda(), torch.from_numpy(ivs).cuda(), torch.from_numpy(ius).cuda()]
    got = got.double().cpu().numpy()
    del out
    want = orc.forward_rays(geo, ang, xh, views, ivs, ius, "interp")
    assert _rel(got, want) < 1e-4, _rel(got, want)


def test_1024_fdk_wang_central_slice_vs_oracle(P, orc, large):
    """FDK with Wang weights at 1024^3 x 1440 on the offset detector, on the
    GPU's full launch, against the oracle at central-slice voxels.  The
    projections are the closed-form line integrals of the head phantom on
    the 16 detector rows around the central row (zero elsewhere): the
    filter works row by row and a central-slice voxel projects between the
    two central rows in every view, so the oracle needs only those 16 rows
    (a detector of 16 rows with the same centre)."""
    geo, ang, plan = large["geo"], large["ang"], large["plan"]
    nv, nu = geo.nDetector
    band = geo.replace(nDetector=(16, nu))
    ells = synth.head_phantom(geo, 3)
    q = orc.analytic_projections(band, ang, ells)           # (1440, 16, nu) FP64
    y = torch.zeros((len(ang), nv, nu), device="cuda")
    y[:, nv // 2 - 8:nv // 2 + 8] = torch.from_numpy(q.astype(np.float32)).cuda()
    rec = P.fdk(plan, y, wang=True)
    del y
    rng = np.random.Generator(np.random.PCG64(85))
    r = rng.uniform(0, 0.85 * geo.nVoxel[2] / 2, 96)
    t = rng.uniform(0, 2 * np.pi, 96)
    ix = np.clip((geo.nVoxel[2] / 2 + r * np.cos(t)).astype(np.int64), 0, geo.nVoxel[2] - 1)
    iy = np.clip((geo.nVoxel[1] / 2 + r * np.sin(t)).astype(np.int64), 0, geo.nVoxel[1] - 1)
    iz = np.full(96, geo.nVoxel[0] // 2)
    got = rec[torch.from_numpy(iz).cuda(), torch.from_numpy(iy).cuda(), torch.from_numpy(ix).cuda()]
    got = got.double().cpu().numpy()
    qf = orc.fdk_filter(band, q.astype(np.float32).astype(np.float64), ntotal=len(ang), wang=True)
    want = orc.bfdk_voxels(band, ang, qf, iz, iy, ix)
    assert _rel(got, want) < 1e-4, _rel(got, want)


def test_1024_siddon_forward_constant_volume_is_box_chord(P, orc, large):
    geo, ang, plan = large["geo"], large["ang"], large["plan"]
    x = torch.ones(geo.nVoxel, device="cuda")
    out = plan.forward(x, kind="siddon")
    rng = np.random.Generator(np.random.PCG64(76))
    n = 1024
    views = np.concatenate([rng.integers(0, len(ang), n - 64), np.full(64, len(ang) - 1)])
    ivs = rng.integers(0, geo.nDetector[0], n)
    ius = rng.integers(0, geo.nDetector[1], n)
    got = out[torch.from_numpy(views).cuda(), torch.from_numpy(ivs).cuda(), torch.from_numpy(ius).cuda()]
    want = _box_chords(geo, ang, views, ivs, ius, orc)
    assert np.max(np.abs(got.double().cpu().numpy() - want)) < 2e-5 * want.max()


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_1024_backward_view_ranges_and_oracle_subset(P, orc, large, kind):
    """A^T over all 1440 views equals the sum of two view ranges (offsets
    past 2^31 in the full call); on the last 8 views the sampled voxels match
    the oracle."""
    geo, ang, plan = large["geo"], large["ang"], large["plan"]
    g = torch.Generator(device="cuda").manual_seed(77)
    y = torch.rand((len(ang),) + geo.nDetector, generator=g, device="cuda")
    # the views the oracle sees come from the seeded host generator
    tail_h = synth.uniform_projections(geo, 8, 76)
    y[-8:] = torch.from_numpy(tail_h).cuda()
    full = plan.backproject(y, kind=kind)
    part = plan.backproject(y[:1000], kind=kind, view0=0, nviews=1000)
    plan.backproject(y[1000:], out=part, kind=kind, beta=1.0, view0=1000, nviews=len(ang) - 1000)
    assert (full - part).norm().item() < 1e-5 * full.norm().item()
    del full, part
    tail = y[-8:].contiguous()
    sub = plan.backproject(tail, kind=kind, view0=len(ang) - 8, nviews=8)
    iz, iy, ix = _fov_voxels(geo, 12, 78)
    got = sub[torch.from_numpy(iz).cuda(), torch.from_numpy(iy).cuda(), torch.from_numpy(ix).cuda()]
    want = orc.adjoint_voxels(geo, ang[-8:], tail_h.astype(np.float64), iz, iy, ix, kind)
    assert _rel(got.double().cpu().numpy(), want) < 1e-4


def test_1024_fdk_backprojector_of_constant(P, large):
    """q == 1: (B q)(X) = N DSO^3 / (DSO^2 - r^2)^(3/2) wherever the bilinear
    footprint stays on the detector."""
    geo, ang, plan = large["geo"], large["ang"], large["plan"]
    q = torch.ones((len(ang),) + geo.nDetector, device="cuda")
    out = plan.backproject(q, kind="fdk")
    iz, iy, ix = _fov_voxels(geo, 64, 79, rmax=0.6)
    iz = iz // 4 + 3 * geo.nVoxel[0] // 8        # central quarter in z
    got = out[torch.from_numpy(iz).cuda(), torch.from_numpy(iy).cuda(), torch.from_numpy(ix).cuda()]
    h = geo.dVoxel[2]
    X = (ix + 0.5 - geo.nVoxel[2] / 2) * h
    Y = (iy + 0.5 - geo.nVoxel[1] / 2) * h
    r2 = X * X + Y * Y
    want = len(ang) * geo.DSO ** 3 / (geo.DSO ** 2 - r2) ** 1.5
    assert np.max(np.abs(got.double().cpu().numpy() / want - 1.0)) < 1e-5


def test_1024_fdk_filter_wang_offset_detector(P, orc, large):
    geo, ang, plan = large["geo"], large["ang"], large["plan"]
    g = torch.Generator(device="cuda").manual_seed(80)
    y = torch.rand((len(ang),) + geo.nDetector, generator=g, device="cuda")
    # the rows the oracle filters come from the seeded host generator
    ref_h = synth.uniform_projections(geo, 2, 81)
    y[:2] = torch.from_numpy(ref_h).cuda()
    ref_in = ref_h.astype(np.float64)
    plan.fdk_filter(y, out=y, wang=True)
    want = orc.fdk_filter(geo, ref_in, ntotal=len(ang), wang=True)
    assert _rel(y[:2].cpu().numpy(), want) < 1e-5
