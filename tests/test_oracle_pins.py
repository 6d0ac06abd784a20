"""Pins of the FP64 oracle to facts fixed by the mathematics, not by itself.

Each test checks the oracle against a closed form, an invariant, a brute
force evaluation on a tiny problem or a textbook/library routine, so that a
dropped term, a wrong sign or index or a transposed operand in the oracle
fails at least one of them.
"""
import math

import numpy as np
import pytest

import synth
from synth import Ellipsoid, Geometry

TINY = Geometry(DSD=60.0, DSO=40.0, nVoxel=(8, 8, 8), dVoxel=(1.0, 1.0, 1.0), nDetector=(10, 12),
                dDetector=(1.7, 1.6), offOrigin=(0.3, -0.4, 0.2), offDetector=(0.5, -0.7))
TINY_ANISO = Geometry(DSD=70.0, DSO=45.0, nVoxel=(6, 8, 7), dVoxel=(1.2, 0.9, 1.1), nDetector=(9, 13),
                      dDetector=(1.5, 1.3), offOrigin=(-0.2, 0.5, 0.1), offDetector=(-0.4, 0.3))


def _angles(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.uniform(0, 2 * np.pi, n))


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


# ------------------------------------------------------- Siddon, brute force
@pytest.mark.parametrize("geo", [TINY, TINY_ANISO])
def test_siddon_equals_cellwise_chords(orc, geo):
    """Siddon's merged-crossing sum equals sum_j chord(ray, cell j) x_j where
    every chord is a separate slab clip of the segment with one cell."""
    ang = _angles(5, 1)
    M = orc.dense_matrix(geo, ang, "siddon")
    x = np.random.Generator(np.random.PCG64(2)).random(geo.nVoxel)
    assert _rel(orc.forward(geo, ang, x, "siddon").ravel(), M @ x.ravel()) < 1e-12
    # every ray's lengths add up to its chord through the volume box
    assert _rel(M.sum(1), orc.forward(geo, ang, np.ones(geo.nVoxel), "siddon").ravel()) < 1e-12


def test_siddon_row_vs_fine_sampling(orc):
    """A matrix row against pure-numpy point sampling of the segment: the
    fraction of 2e5 equispaced points falling into each cell times |P - S|."""
    geo = TINY
    ang = _angles(2, 3)
    M = orc.dense_matrix(geo, ang, "siddon")
    nz, ny, nx = geo.nVoxel
    lo = np.array([geo.offOrigin[2] - nx * geo.dVoxel[2] / 2, geo.offOrigin[1] - ny * geo.dVoxel[1] / 2,
                   geo.offOrigin[0] - nz * geo.dVoxel[0] / 2])
    h = np.array([geo.dVoxel[2], geo.dVoxel[1], geo.dVoxel[0]])
    npts = 200000
    for k, iv, iu in [(0, 4, 5), (1, 2, 8), (0, 7, 3)]:
        S, P = orc.ray_endpoints(geo, ang[k], iv, iu)
        t = (np.arange(npts) + 0.5) / npts
        X = S[None, :] + t[:, None] * (P - S)[None, :]
        idx = np.floor((X - lo) / h).astype(int)
        ok = np.all((idx >= 0) & (idx < np.array([nx, ny, nz])), 1)
        lin = (idx[ok, 2] * ny + idx[ok, 1]) * nx + idx[ok, 0]
        row = np.bincount(lin, minlength=geo.n_vox) * np.linalg.norm(P - S) / npts
        r = (k * geo.nDetector[0] + iv) * geo.nDetector[1] + iu
        assert np.max(np.abs(row - M[r])) < 2e-3
        assert row.sum() > 1.0


def _box_chord_np(S, P, bl, bh):
    d = P - S
    L = np.linalg.norm(d, axis=-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        a_lo = (bl - S) / d
        a_hi = (bh - S) / d
    a0 = np.max(np.minimum(a_lo, a_hi), axis=-1)
    a1 = np.min(np.maximum(a_lo, a_hi), axis=-1)
    a0 = np.maximum(a0, 0.0)
    a1 = np.minimum(a1, 1.0)
    return np.where(a1 > a0, (a1 - a0) * L, 0.0)


def test_siddon_cuboid_phantom_exact(orc):
    """Unions of whole voxels with constant densities: the ray sum is exactly
    sum_b rho_b * (chord through block b), at any grid size."""
    geo = Geometry(DSD=150.0, DSO=100.0, nVoxel=(24, 20, 22), dVoxel=(1.1, 0.9, 1.0), nDetector=(30, 40),
                   dDetector=(1.3, 1.2), offOrigin=(0.4, -0.7, 0.9), offDetector=(0.6, -1.1))
    ang = _angles(6, 5)
    rng = np.random.Generator(np.random.PCG64(6))
    x = np.zeros(geo.nVoxel)
    blocks = []
    for _ in range(5):
        i0 = [int(rng.integers(0, n - 3)) for n in geo.nVoxel]
        i1 = [int(rng.integers(a + 1, n + 1)) for a, n in zip(i0, geo.nVoxel)]
        rho = float(rng.uniform(0.2, 1.0))
        x[i0[0]:i1[0], i0[1]:i1[1], i0[2]:i1[2]] += rho
        blocks.append((i0, i1, rho))
    blocks.append(([0, 0, 0], list(geo.nVoxel), 0.05))   # the whole volume (x == 1 case)
    x += 0.05
    p = orc.forward(geo, ang, x, "siddon")
    nz, ny, nx = geo.nVoxel
    dz, dy, dx = geo.dVoxel
    oz, oy, ox = geo.offOrigin
    lo = np.array([ox - nx * dx / 2, oy - ny * dy / 2, oz - nz * dz / 2])
    h = np.array([dx, dy, dz])
    nv, nu = geo.nDetector
    ref = np.zeros_like(p)
    for k in range(len(ang)):
        SP = [orc.ray_endpoints(geo, ang[k], iv, iu) for iv in range(nv) for iu in range(nu)]
        S = np.array([a for a, _ in SP])
        P = np.array([b for _, b in SP])
        acc = np.zeros(len(SP))
        for i0, i1, rho in blocks:
            bl = lo + np.array([i0[2], i0[1], i0[0]]) * h
            bh = lo + np.array([i1[2], i1[1], i1[0]]) * h
            acc += rho * _box_chord_np(S, P, bl, bh)
        ref[k] = acc.reshape(nv, nu)
    assert np.max(np.abs(p - ref)) < 1e-10 * np.max(np.abs(ref))


# ------------------------------------------------- interpolated, brute force
@pytest.mark.parametrize("geo", [TINY, TINY_ANISO])
def test_interp_equals_explicit_tent_matrix(orc, geo):
    """Trilinear ray marching equals the matrix whose entries evaluate the
    tent phi(c - j) directly for every (sample, voxel) pair."""
    ang = _angles(5, 7)
    M = orc.dense_matrix(geo, ang, "interp")
    x = np.random.Generator(np.random.PCG64(8)).random(geo.nVoxel)
    assert _rel(orc.forward(geo, ang, x, "interp").ravel(), M @ x.ravel()) < 1e-12
    y = np.random.Generator(np.random.PCG64(9)).random((len(ang),) + geo.nDetector)
    assert _rel(orc.backward(geo, ang, y, "interp").ravel(), M.T @ y.ravel()) < 1e-12


def test_interp_sample_phase_anchored_at_source(orc):
    """Samples sit at t_k = k ds from the source: moving the volume along an
    oblique ray by a whole number of steps leaves that ray's sum unchanged,
    and by a fraction of a step changes it."""
    geo = Geometry(DSD=150.0, DSO=100.0, nVoxel=(8, 8, 8), dVoxel=(1.0, 1.0, 1.0), nDetector=(1, 1),
                   dDetector=(1.0, 1.0), offDetector=(2.3, 3.1))
    x = np.random.Generator(np.random.PCG64(10)).random(geo.nVoxel)
    ang = np.array([0.3])
    S, P = orc.ray_endpoints(geo, ang[0], 0.0, 0.0)
    dh = (P - S) / np.linalg.norm(P - S)
    p0 = orc.forward(geo, ang, x, "interp")[0, 0, 0]
    assert p0 > 1.0
    ds = geo.accuracy * 1.0
    for shift in (ds * 3, -ds * 5):
        g2 = geo.replace(offOrigin=tuple(shift * dh[::-1]))
        assert abs(orc.forward(g2, ang, x, "interp")[0, 0, 0] - p0) < 1e-11 * abs(p0)
    g3 = geo.replace(offOrigin=tuple(0.3 * ds * dh[::-1]))
    assert abs(orc.forward(g3, ang, x, "interp")[0, 0, 0] - p0) > 1e-5 * abs(p0)


# ----------------------------------------------------- transposes / adjoints
@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_dot_product_identity(orc, kind):
    geo = Geometry(DSD=150.0, DSO=100.0, nVoxel=(20, 24, 22), dVoxel=(1.0, 1.1, 0.9), nDetector=(28, 36),
                   dDetector=(1.4, 1.3), offOrigin=(0.5, 0.2, -0.3), offDetector=(0.7, -0.4))
    ang = _angles(9, 11)
    rng = np.random.Generator(np.random.PCG64(12))
    x = rng.random(geo.nVoxel)
    y = rng.random((len(ang),) + geo.nDetector)
    lhs = np.vdot(orc.forward(geo, ang, x, kind), y)
    rhs = np.vdot(x, orc.backward(geo, ang, y, kind))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_scatter_transpose_equals_per_voxel_bruteforce(orc, kind):
    """The ray-driven scatter A^T y against per-voxel brute force over each
    voxel's detector footprint (different loop order, independent code)."""
    geo = Geometry(DSD=150.0, DSO=100.0, nVoxel=(18, 20, 16), dVoxel=(1.0, 1.0, 1.2), nDetector=(26, 30),
                   dDetector=(1.4, 1.3), offOrigin=(0.3, -0.2, 0.4), offDetector=(-0.6, 0.8))
    ang = _angles(7, 13)
    rng = np.random.Generator(np.random.PCG64(14))
    y = rng.random((len(ang),) + geo.nDetector)
    bt = orc.backward(geo, ang, y, kind)
    sel = rng.integers(0, geo.n_vox, 300)
    iz, iy, ix = np.unravel_index(sel, geo.nVoxel)
    bf = orc.adjoint_voxels(geo, ang, y, iz, iy, ix, kind)
    assert _rel(bf, bt.ravel()[sel]) < 1e-12


# -------------------------------------------------------------- equivariance
@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_rotation_and_flip_equivariance(orc, kind):
    """Rotating the object by +90 deg about z equals shifting the view index
    by -N/4; flipping z equals flipping the detector's v axis."""
    geo = Geometry(DSD=150.0, DSO=100.0, nVoxel=(14, 16, 16), dVoxel=(1.0, 1.0, 1.0), nDetector=(20, 26),
                   dDetector=(1.2, 1.3), offDetector=(0.0, 0.45))
    N = 8
    ang = synth.circular_angles(N)
    x = np.random.Generator(np.random.PCG64(15)).random(geo.nVoxel)
    n = geo.nVoxel[2]
    # new(X, Y) = old(Y, -X): new[:, iy, ix] = old[:, n - 1 - ix, iy]
    iy, ix = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    xr = x[:, n - 1 - ix, iy]
    p = orc.forward(geo, ang, x, kind)
    pr = orc.forward(geo, ang, xr, kind)
    assert _rel(pr, np.roll(p, N // 4, axis=0)) < 1e-12
    assert _rel(pr, p) > 1e-3
    pz = orc.forward(geo, ang, x[::-1], kind)
    assert _rel(pz, p[:, ::-1, :]) < 1e-12


# ------------------------------------------------------ continuum convergence
def _phantom_64mm():
    g = Geometry(DSD=1536.0, DSO=1000.0, nVoxel=(64, 64, 64), dVoxel=(1.0, 1.0, 1.0), nDetector=(48, 48),
                 dDetector=(2.0, 2.0))
    return synth.random_ellipsoids(g, seed=21, count_range=(6, 8), axis_range=(6.0, 18.0))


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_ellipsoid_closed_form_convergence(orc, kind):
    """Projections of the voxelised phantom converge to the closed-form line
    integrals as the grid is refined (same physical object and detector)."""
    ell = _phantom_64mm()
    ang = _angles(6, 22)
    errs = []
    for n in (16, 32, 64):
        d = 64.0 / n
        geo = Geometry(DSD=1536.0, DSO=1000.0, nVoxel=(n, n, n), dVoxel=(d, d, d), nDetector=(48, 48),
                       dDetector=(2.0, 2.0))
        x = synth.voxelize(geo, ell, sub=4, dtype=np.float64)
        p = orc.forward(geo, ang, x, kind)
        pa = orc.analytic_projections(geo, ang, ell)
        errs.append(_rel(p, pa))
    order = math.log2(errs[0] / errs[2]) / 2
    assert errs[0] > errs[1] > errs[2]
    assert order >= 0.8, (errs, order)
    assert errs[2] < 0.06


def test_ellipsoid_chord_closed_form():
    import oracle
    rng = np.random.Generator(np.random.PCG64(23))
    e = Ellipsoid((1.0, -2.0, 0.5), (7.0, 4.0, 5.0), tuple(map(tuple, np.linalg.qr(rng.normal(size=(3, 3)))[0])), 1.0)
    npts = 400000
    for _ in range(4):
        S = rng.normal(size=3) * 3 + np.array([40.0, 0, 0])
        P = rng.normal(size=3) * 3 + np.array([-40.0, 0, 0])
        t = (np.arange(npts) + 0.5) / npts
        X = S + t[:, None] * (P - S)
        q = ((X - np.array(e.c)) @ np.array(e.R)) / np.array(e.a)
        quad = np.mean(np.sum(q * q, 1) <= 1.0) * np.linalg.norm(P - S)
        cf = oracle.ellipsoid_line_integrals([e], S[None], P[None])[0]
        assert abs(cf - quad) < 1e-3
    # a sphere: chord 2 sqrt(r^2 - d^2) at distance d from the centre
    sph = Ellipsoid((0.0, 0.0, 0.0), (5.0, 5.0, 5.0), ((1, 0, 0), (0, 1, 0), (0, 0, 1)), 2.0)
    for dd in (0.0, 1.5, 4.9, 5.1):
        S = np.array([[30.0, dd, 0.0]])
        P = np.array([[-30.0, dd, 0.0]])
        want = 2.0 * 2.0 * math.sqrt(max(25.0 - dd * dd, 0.0))
        assert abs(oracle.ellipsoid_line_integrals([sph], S, P)[0] - want) < 1e-12


# ------------------------------------------------------------------- FDK
def _ball(r, c=(0.0, 0.0, 0.0), rho=1.0):
    return Ellipsoid(c, (r, r, r), ((1, 0, 0), (0, 1, 0), (0, 0, 1)), rho)


def test_fdk_uniform_ball(orc):
    """A uniform unit-density ball reconstructs to 1 in its interior (FDK
    scaling: cosine weight, Ram-Lak ramp, angular factor, (DSO/U)^2)."""
    geo, _ = synth.workload("head64")
    ang = synth.circular_angles(128)
    R = 0.6 * geo.iso_fov_radius()
    pa = orc.analytic_projections(geo, ang, [_ball(R)])
    f = orc.fdk(geo, ang, pa)
    nz, ny, nx = geo.nVoxel
    yc = (np.arange(ny) + 0.5 - ny / 2)
    xc = (np.arange(nx) + 0.5 - nx / 2)
    r2 = yc[:, None] ** 2 + xc[None, :] ** 2
    mid = f[nz // 2 - 1:nz // 2 + 1]
    interior = mid[:, r2 < (0.8 * R) ** 2]
    assert abs(interior.mean() - 1.0) < 0.01, interior.mean()
    outside = mid[:, r2 > (1.2 * R) ** 2]
    assert abs(outside.mean()) < 0.02


def test_fdk_off_centre_ball_lands_in_place(orc):
    """The reconstructed centroid of an off-centre ball is the ball centre:
    the backprojector's detector mapping agrees with the ray geometry."""
    geo, _ = synth.workload("head64")
    geo = geo.replace(offOrigin=(1.5, -2.0, 3.0), offDetector=(0.8, -1.3))
    ang = synth.circular_angles(96)
    c = (9.0 + 3.0, -6.0 - 2.0, 4.0 + 1.5)
    pa = orc.analytic_projections(geo, ang, [_ball(7.0, c)])
    f = orc.fdk(geo, ang, pa)
    f = np.where(f > 0.5, f, 0.0)
    nz, ny, nx = geo.nVoxel
    Z, Y, X = np.meshgrid((np.arange(nz) + 0.5 - nz / 2) + 1.5, (np.arange(ny) + 0.5 - ny / 2) - 2.0,
                          (np.arange(nx) + 0.5 - nx / 2) + 3.0, indexing="ij")
    m = f.sum()
    cen = ((f * X).sum() / m, (f * Y).sum() / m, (f * Z).sum() / m)
    assert np.allclose(cen, c, atol=0.15), cen


def test_ramp_filter_frequency_response(orc):
    """The Ram-Lak kernel is the band-limited ramp: a row cos(2 pi f u) is
    returned scaled by |f| (away from the row ends), times the FDK angular
    factor pi/N.  The geometry makes the cosine weight 1 to 1e-12."""
    nu = 2048
    geo = Geometry(DSD=2e7, DSO=1e7, nVoxel=(4, 4, 4), dVoxel=(1.0, 1.0, 1.0), nDetector=(1, nu),
                   dDetector=(1.0, 1.0))
    tau = geo.dDetector[1] * geo.DSO / geo.DSD
    N = 7
    u = (np.arange(nu) + 0.5 - nu / 2) * tau
    for f in (0.02, 0.11, 0.37, 0.93):           # cycles per mm at iso (Nyquist = 1 / (2 tau) = 1)
        row = np.cos(2 * np.pi * f * u)
        out = orc.fdk_filter(geo, np.tile(row, (N, 1, 1)), ntotal=N)[0, 0]
        centre = slice(nu // 2 - 64, nu // 2 + 64)
        want = abs(f) * row * (np.pi / N)
        assert np.max(np.abs(out[centre] - want[centre])) < 2e-3 * (np.pi / N), f
    # DC: the ramp removes the mean of a long constant row (up to the 1/n tail)
    out = orc.fdk_filter(geo, np.ones((N, 1, nu)), ntotal=N)[0, 0]
    assert abs(out[nu // 2]) < 1e-3 * (np.pi / N)


def test_bfdk_constant_closed_form(orc):
    """q == 1 on the detector: (B q)(X) = sum_k (DSO / (DSO - r cos(theta_k - phi)))^2,
    which for N uniform views is N DSO^3 / (DSO^2 - r^2)^(3/2)."""
    geo = Geometry(DSD=300.0, DSO=200.0, nVoxel=(6, 20, 20), dVoxel=(2.0, 2.0, 2.0), nDetector=(80, 120),
                   dDetector=(1.5, 1.5))
    N = 48
    ang = synth.circular_angles(N)
    out = orc.bfdk(geo, ang, np.ones((N,) + geo.nDetector))
    yc = (np.arange(20) + 0.5 - 10) * 2.0
    xc = (np.arange(20) + 0.5 - 10) * 2.0
    r2 = yc[:, None] ** 2 + xc[None, :] ** 2
    want = N * geo.DSO ** 3 / (geo.DSO ** 2 - r2) ** 1.5
    assert np.max(np.abs(out / want[None] - 1.0)) < 1e-12


def test_bfdk_impulse_matches_ray_geometry(orc):
    """A single-pixel impulse backprojects onto voxel X with weight
    (DSO/U)^2 * bilinear hat, where the detector position of X is found by
    intersecting the line S-X with the detector plane spanned by the ray
    end points (no formula shared with the oracle's backprojector)."""
    geo = Geometry(DSD=300.0, DSO=200.0, nVoxel=(6, 8, 10), dVoxel=(2.0, 2.0, 2.0), nDetector=(40, 50),
                   dDetector=(1.5, 1.5), offOrigin=(1.0, -2.0, 3.0), offDetector=(0.7, -0.9))
    th = 0.7
    nz, ny, nx = geo.nVoxel
    S, P00 = orc.ray_endpoints(geo, th, 0.0, 0.0)
    _, P01 = orc.ray_endpoints(geo, th, 0.0, 1.0)
    _, P10 = orc.ray_endpoints(geo, th, 1.0, 0.0)
    eu, ev = P01 - P00, P10 - P00
    rng = np.random.Generator(np.random.PCG64(31))
    for _ in range(6):
        iz, iy, ix = int(rng.integers(nz)), int(rng.integers(ny)), int(rng.integers(nx))
        X = np.array([3.0 - nx + 2.0 * ix + 1.0, -2.0 - ny + 2.0 * iy + 1.0, 1.0 - nz + 2.0 * iz + 1.0])
        # solve S + t (X - S) = P00 + a eu + b ev
        A = np.stack([X - S, -eu, -ev], 1)
        t, fu, fv = np.linalg.solve(A, P00 - S)
        iu, ivv = int(np.floor(fu)), int(np.floor(fv))
        q = np.zeros((1,) + geo.nDetector)
        q[0, ivv, iu] = 1.0
        out = orc.bfdk(geo, np.array([th]), q)[iz, iy, ix]
        nrm = np.cross(eu, ev)
        U = np.dot(X - S, nrm) / np.dot(P00 - S, nrm) * geo.DSD    # distance along the axis
        want = (geo.DSO * geo.DSD / U / geo.DSD) ** 2 * (1 - (fu - iu)) * (1 - (fv - ivv))
        assert abs(out - want) < 1e-12 * max(want, 1e-3), (out, want)


def test_wang_weight_partition_of_unity(orc):
    geo, _ = synth.workload("large1024")
    D = geo.nDetector[1] * geo.dDetector[1] / 2 - abs(geo.offDetector[1])
    for u in np.linspace(-D, D, 41):
        assert abs(orc.wang_weight(geo, u) + orc.wang_weight(geo, -u) - 1.0) < 1e-14
    assert orc.wang_weight(geo, D + 1.0) == 1.0
    assert orc.wang_weight(geo, -D - 1.0) == 0.0
    assert abs(orc.wang_weight(geo, 0.0) - 0.5) < 1e-15


def test_fdk_wang_offset_detector_ball(orc):
    """Offset detector that sees only part of a ball in each view (shadow
    half-width 40 mm, detector u in [-32.8, 56.8] mm): FDK with Wang weights
    still reconstructs the unit density; without them it does not."""
    geo = Geometry(DSD=1536.0, DSO=1000.0, nVoxel=(8, 64, 64), dVoxel=(1.0, 1.0, 1.0), nDetector=(16, 56),
                   dDetector=(1.6, 1.6), offDetector=(0.0, 12.0))
    ang = synth.circular_angles(180)
    R = 26.0
    pa = orc.analytic_projections(geo, ang, [_ball(R)])
    f = orc.fdk(geo, ang, pa, wang=True)
    yc = (np.arange(64) + 0.5 - 32)
    r2 = yc[:, None] ** 2 + yc[None, :] ** 2
    interior = f[3:5][:, r2 < (0.8 * R) ** 2]
    assert abs(interior.mean() - 1.0) < 0.015, interior.mean()
    nowang = orc.fdk(geo, ang, pa, wang=False)[3:5][:, r2 < (0.8 * R) ** 2]
    assert abs(nowang.mean() - 1.0) > 0.05


# ------------------------------------------------------------------ CGLS
def _krylov_solutions(M, b, kmax):
    """x_k = argmin_{x in K_k(M^T M, M^T b)} |M x - b|, orthonormal basis by
    modified Gram-Schmidt (twice), then a dense least-squares solve."""
    n = M.shape[1]
    V = np.zeros((n, 0))
    v = M.T @ b
    sols = []
    for _ in range(kmax):
        for _ in range(2):
            v = v - V @ (V.T @ v)
        v = v / np.linalg.norm(v)
        V = np.concatenate([V, v[:, None]], 1)
        c, *_ = np.linalg.lstsq(M @ V, b, rcond=None)
        sols.append(V @ c)
        v = M.T @ (M @ v)
    return sols


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_cgls_iterates_are_krylov_minimisers(orc, kind):
    geo = Geometry(DSD=60.0, DSO=40.0, nVoxel=(8, 8, 8), dVoxel=(1.0, 1.0, 1.0), nDetector=(8, 8),
                   dDetector=(1.6, 1.6))
    ang = synth.circular_angles(8)
    rng = np.random.Generator(np.random.PCG64(41))
    xt = rng.random(geo.nVoxel)
    M = orc.dense_matrix(geo, ang, kind)
    b = M @ xt.ravel() + 0.01 * rng.standard_normal(M.shape[0])
    ref = _krylov_solutions(M, b, 8)
    for k in range(1, 9):
        xk, hist = orc.cgls(geo, ang, b.reshape((8,) + geo.nDetector), k, kind)
        assert _rel(xk.ravel(), ref[k - 1]) < 1e-8, k
    _, hist = orc.cgls(geo, ang, b.reshape((8,) + geo.nDetector), 12, kind, x_gt=xt)
    res = hist["resid"]
    assert all(res[i + 1] <= res[i] * (1 + 1e-12) for i in range(len(res) - 1))


def _missing_rays_problem():
    """A detector much wider than the volume's shadow, with data only on
    columns whose rays miss the volume: A^T b = 0."""
    geo = Geometry(DSD=60.0, DSO=40.0, nVoxel=(8, 8, 8), dVoxel=(1.0, 1.0, 1.0), nDetector=(8, 40),
                   dDetector=(1.6, 1.6))
    ang = synth.circular_angles(4)
    b = np.zeros((4,) + geo.nDetector)
    b[:, :, :4] = 1.0
    b[:, :, -4:] = 2.0
    return geo, ang, b


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_cgls_breakdown_stops_at_once(orc, kind):
    """CGLS breakdown (gamma = |A^T r|^2 = 0 before the first step): the run
    stops at iteration 0 with the flag set and x = 0, for b = 0 and for data
    the operator's range cannot see (rays that miss the volume; checked with
    the dense matrix).  A step taken anyway would divide 0 by 0."""
    geo, ang, b = _missing_rays_problem()
    M = orc.dense_matrix(geo, ang, kind)
    assert np.all(M[b.ravel() != 0] == 0) and np.any(M != 0)
    for data in (np.zeros_like(b), b):
        x, hist = orc.cgls(geo, ang, data, 5, kind)
        assert hist["stopped"] == 0 and hist["resid"] == [] and not np.any(x)


def test_cgls_norm_of_iterate_grows(orc):
    geo = Geometry(DSD=60.0, DSO=40.0, nVoxel=(8, 8, 8), dVoxel=(1.0, 1.0, 1.0), nDetector=(8, 8),
                   dDetector=(1.6, 1.6))
    ang = synth.circular_angles(6)
    b = np.random.Generator(np.random.PCG64(42)).random((6, 8, 8))
    norms = [np.linalg.norm(orc.cgls(geo, ang, b, k, "siddon")[0]) for k in range(1, 8)]
    assert all(norms[i + 1] >= norms[i] * (1 - 1e-12) for i in range(len(norms) - 1))


# --------------------------------------------------------------- OS-SART
@pytest.mark.parametrize("blocksize", [1, 4, 12])
def test_os_sart_converges_on_consistent_data(orc, blocksize):
    """On noise-free data of a non-negative image, SART (blocksize 1),
    OS-SART and SIRT (one block) drive the residual down monotonically per
    pass, and the true image is a fixed point."""
    geo = Geometry(DSD=60.0, DSO=40.0, nVoxel=(6, 6, 6), dVoxel=(1.0, 1.0, 1.0), nDetector=(8, 8),
                   dDetector=(1.4, 1.4))
    ang = synth.circular_angles(12)
    xt = np.random.Generator(np.random.PCG64(43)).random(geo.nVoxel)
    b = orc.forward(geo, ang, xt, "interp")
    res = []
    x = None
    for it in range(6):
        x = orc.os_sart(geo, ang, b, 1, blocksize, x0=x, kind="interp")
        res.append(np.linalg.norm(orc.forward(geo, ang, x, "interp") - b))
    assert all(res[i + 1] < res[i] for i in range(len(res) - 1)), res
    assert res[-1] < 0.5 * res[0]
    xf = orc.os_sart(geo, ang, b, 1, blocksize, x0=xt, kind="interp")
    assert _rel(xf, xt) < 1e-12


def test_sirt_one_block_one_pass_is_weighted_gradient_step(orc):
    """With one block the update is x1 = lam V (A^T W b) from x0 = 0, i.e. a
    step along A^T W b -- checked through the dense matrix."""
    geo = Geometry(DSD=60.0, DSO=40.0, nVoxel=(6, 6, 6), dVoxel=(1.0, 1.0, 1.0), nDetector=(8, 8),
                   dDetector=(1.4, 1.4))
    ang = synth.circular_angles(5)
    M = orc.dense_matrix(geo, ang, "siddon")
    b = np.random.Generator(np.random.PCG64(44)).random(M.shape[0])
    row = M.sum(1)
    col = M.sum(0)
    W = np.where(row > 0, 1 / np.where(row > 0, row, 1), 0)
    V = np.where(col > 0, 1 / np.where(col > 0, col, 1), 0)
    want = 0.7 * V * (M.T @ (W * b))
    got = orc.os_sart(geo, ang, b.reshape((5,) + geo.nDetector), 1, 5, lam=0.7, nonneg=False, kind="siddon")
    assert _rel(got.ravel(), want) < 1e-12


# ------------------------------------------------------- general geometry
_GG = Geometry(DSD=60.0, DSO=40.0, nVoxel=(8, 8, 8), dVoxel=(1.0, 1.0, 1.0), nDetector=(10, 10),
               dDetector=(1.3, 1.3))


def _rand8(seed):
    return np.random.Generator(np.random.PCG64(seed)).random((8, 8, 8))


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_views_default_equals_circular(orc, kind):
    """ZYZ angles (theta, 0, 0) with the geometry's own parameters are the
    circular orbit (offsets included)."""
    geo = Geometry(DSD=60.0, DSO=40.0, nVoxel=(8, 9, 7), dVoxel=(1.0, 1.1, 0.9), nDetector=(10, 12),
                   dDetector=(1.3, 1.2), offOrigin=(0.3, -0.2, 0.5), offDetector=(0.4, -0.7))
    ang = synth.circular_angles(5) + 0.1
    x = np.random.Generator(np.random.PCG64(53)).random(geo.nVoxel)
    y = np.random.Generator(np.random.PCG64(54)).random((5,) + geo.nDetector)
    v = synth.views(geo, ang)
    assert _rel(orc.forward(geo, v, x, kind), orc.forward(geo, ang, x, kind)) < 1e-13
    assert _rel(orc.backward(geo, v, y, kind), orc.backward(geo, ang, y, kind)) < 1e-13


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_detector_half_turns_flip_the_image(orc, kind):
    """A centred detector rolled by pi (about its normal) sees the image
    flipped in u and v; yawed by pi (about v) flipped in u; pitched by pi
    (about u) flipped in v."""
    ang = synth.circular_angles(4) + 0.3
    x = _rand8(55)
    p = orc.forward(_GG, ang, x, kind)
    roll = orc.forward(_GG, synth.views(_GG, ang, rotDetector=(np.pi, 0.0, 0.0)), x, kind)
    pitch = orc.forward(_GG, synth.views(_GG, ang, rotDetector=(0.0, np.pi, 0.0)), x, kind)
    yaw = orc.forward(_GG, synth.views(_GG, ang, rotDetector=(0.0, 0.0, np.pi)), x, kind)
    assert _rel(roll, p[:, ::-1, ::-1]) < 1e-12
    assert _rel(pitch, p[:, ::-1, :]) < 1e-12
    assert _rel(yaw, p[:, :, ::-1]) < 1e-12


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_detector_quarter_roll_transposes_square_detector(orc, kind):
    """Rolled by pi/2, the detector's u axis takes the default v direction
    and its v axis the default -u: p_roll[iv, iu] = p[iu, nu - 1 - iv]."""
    ang = synth.circular_angles(3) + 0.2
    x = _rand8(56)
    p = orc.forward(_GG, ang, x, kind)
    q = orc.forward(_GG, synth.views(_GG, ang, rotDetector=(np.pi / 2, 0.0, 0.0)), x, kind)
    want = np.transpose(p, (0, 2, 1))[:, ::-1, :]
    assert _rel(q, want) < 1e-12


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_cor_equals_per_view_origin_shift(orc, kind):
    """Shifting the source-detector line by c along the rotated y axis
    (-sin t, cos t, 0) is the same as moving the volume by -c along it."""
    ang = np.array([0.4, 1.9, 3.3])
    c = 0.7
    x = _rand8(57)
    shift = np.stack([np.zeros(3), -c * np.cos(ang), c * np.sin(ang)], axis=1)   # (z, y, x)
    a = orc.forward(_GG, synth.views(_GG, ang, COR=c), x, kind)
    b = orc.forward(_GG, synth.views(_GG, ang, offOrigin=shift), x, kind)
    assert _rel(a, b) < 1e-12


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_zyz_tilted_orbit_equals_rotated_volume(orc, kind):
    """Gantry (0, pi/2, t): R = Ry(pi/2) Rz(t) maps the circular orbit into
    the y-z plane.  Projecting x this way equals the circular projection of
    x(R_y p), which on a centred cube of isotropic voxels is the index map
    x'[iz, iy, ix] = x[n - 1 - ix, iy, iz]."""
    ang = synth.circular_angles(4) + 0.25
    x = _rand8(58)
    zyz = np.stack([np.zeros(4), np.full(4, np.pi / 2), ang], axis=1)
    a = orc.forward(_GG, synth.views(_GG, zyz), x, kind)
    xr = np.transpose(x[::-1, :, :], (2, 1, 0))
    b = orc.forward(_GG, ang, xr, kind)
    assert _rel(a, b) < 1e-12


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_per_view_distances_and_general_adjoint(orc, kind):
    """Per-view DSO/DSD and offsets equal the views projected one geometry at
    a time; the scatter adjoint stays the exact transpose (dot-product
    identity) under a general geometry."""
    ang = np.array([0.1, 1.3, 2.9, 4.2])
    rng = np.random.Generator(np.random.PCG64(59))
    dso = np.array([38.0, 41.0, 40.0, 44.0])
    dsd = dso + np.array([19.0, 22.0, 20.0, 25.0])
    v = synth.views(_GG, ang, DSO=dso, DSD=dsd, COR=rng.uniform(-0.5, 0.5, 4),
                    offDetector=rng.uniform(-0.6, 0.6, (4, 2)), rotDetector=rng.uniform(-0.2, 0.2, (4, 3)))
    x = _rand8(60)
    full = orc.forward(_GG, v, x, kind)
    for k in range(4):
        one = orc.forward(_GG, v[k:k + 1], x, kind)
        assert _rel(one[0], full[k]) < 1e-14
    y = rng.random(full.shape)
    lhs = float(np.sum(full * y))
    rhs = float(np.sum(x * orc.backward(_GG, v, y, kind)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    vox = orc.adjoint_voxels(_GG, v, y, [1, 4, 6], [2, 5, 3], [7, 0, 4], kind)
    full_bp = orc.backward(_GG, v, y, kind)
    assert _rel(vox, full_bp[[1, 4, 6], [2, 5, 3], [7, 0, 4]]) < 1e-12


# ------------------------------------------------------------ MLEM / OSEM
_EMGEO = Geometry(DSD=60.0, DSO=40.0, nVoxel=(6, 6, 6), dVoxel=(1.0, 1.0, 1.0), nDetector=(8, 8),
                  dDetector=(1.4, 1.4))


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_mlem_preserves_counts(orc, kind):
    """After one EM update the model's total counts equal the data's over
    the rays the model reaches: sum_i (A x1)_i = sum_{i: (A x0)_i > 0} b_i
    (the sensitivity normalisation cancels; a dropped or misplaced
    normaliser breaks it)."""
    geo, ang = _EMGEO, synth.circular_angles(10)
    rng = np.random.Generator(np.random.PCG64(46))
    x0 = 0.5 + rng.random(geo.nVoxel)
    b = rng.random((10,) + geo.nDetector) * 3.0
    x1 = orc.osem(geo, ang, b, 1, x0=x0, kind=kind)
    ax0 = orc.forward(geo, ang, x0, kind)
    want = float(b[ax0 > 0].sum())
    got = float(orc.forward(geo, ang, x1, kind).sum())
    assert abs(got - want) <= 1e-12 * want


@pytest.mark.parametrize("blocksize", [None, 3])
def test_mlem_osem_fixed_point_on_consistent_data(orc, blocksize):
    """With b = A x_t and x_t > 0, x_t is a fixed point of MLEM and OSEM."""
    geo, ang = _EMGEO, synth.circular_angles(12)
    xt = 0.2 + np.random.Generator(np.random.PCG64(47)).random(geo.nVoxel)
    b = orc.forward(geo, ang, xt, "interp")
    x = orc.osem(geo, ang, b, 1, blocksize=blocksize, x0=xt, kind="interp")
    # voxels no ray reaches are set to 0 by the update
    seen = orc.backward(geo, ang, np.ones((12,) + geo.nDetector), "interp") > 0
    assert _rel(x[seen], xt[seen]) < 1e-12
    assert np.all(x[~seen] == 0.0)


def test_mlem_loglik_increases_and_stays_positive(orc):
    """EM never decreases the Poisson log-likelihood (Dempster-Laird-Rubin;
    Shepp-Vardi for emission/transmission counts) and keeps x >= 0."""
    geo, ang = _EMGEO, synth.circular_angles(10)
    rng = np.random.Generator(np.random.PCG64(48))
    xt = rng.random(geo.nVoxel)
    b = rng.poisson(20.0 * orc.forward(geo, ang, xt, "siddon")) / 20.0
    x = None
    ll = []
    for _ in range(8):
        x = orc.osem(geo, ang, b, 1, x0=x, kind="siddon")
        assert np.all(x >= 0.0)
        ll.append(orc.poisson_loglik(geo, ang, b, x, "siddon"))
    assert all(ll[i + 1] >= ll[i] - 1e-9 * abs(ll[i]) for i in range(len(ll) - 1)), ll
    assert ll[-1] > ll[0]


def test_osem_one_block_equals_mlem_and_blocks_differ(orc):
    geo, ang = _EMGEO, synth.circular_angles(12)
    b = np.random.Generator(np.random.PCG64(49)).random((12,) + geo.nDetector)
    m = orc.osem(geo, ang, b, 2, kind="interp")
    o = orc.osem(geo, ang, b, 2, blocksize=12, kind="interp")
    assert _rel(o, m) < 1e-14
    o4 = orc.osem(geo, ang, b, 2, blocksize=4, kind="interp")
    assert _rel(o4, m) > 1e-3


# ------------------------------------------------------- TV / ASD-POCS
def test_tv_of_voxel_aligned_cube_closed_form(orc):
    """Isotropic TV (backward differences, eps = 0) of a cube of side m and
    height h in a zero background: the three upper faces give h per face
    voxel (3 m^2), the lower faces h per voxel on one face (3 (m-1)^2),
    sqrt(2) h on an edge (3 (m-1)) and sqrt(3) h at the corner."""
    m, h = 5, 1.5
    x = np.zeros((12, 13, 11))
    x[3:3 + m, 4:4 + m, 2:2 + m] = h
    want = h * (3 * m * m + 3 * (m - 1) ** 2 + 3 * math.sqrt(2) * (m - 1) + math.sqrt(3))
    assert abs(orc.awtv(x) - want) < 1e-12 * want


def test_awtv_limits(orc):
    """delta -> inf gives plain TV; delta far below the cube's jump switches
    its edges off (weights exp(-(h/delta)^2))."""
    x = np.zeros((10, 10, 10))
    x[2:7, 3:8, 2:6] = 2.0
    assert abs(orc.awtv(x, delta=1e9) - orc.awtv(x)) < 1e-12 * orc.awtv(x)
    assert orc.awtv(x, delta=0.1) < 1e-80


@pytest.mark.parametrize("delta", [math.inf, 0.35])
def test_awtv_gradient_matches_finite_differences(orc, delta):
    """Central differences of sum sqrt(sum_a w_a d_a(y)^2 + eps) at y = x,
    the weights held at x's values, equal awtv_grad(x) (a dropped
    neighbour term, a wrong sign or index fails this)."""
    rng = np.random.Generator(np.random.PCG64(50))
    x = rng.random((5, 6, 7))
    eps = 1e-6
    g = orc.awtv_grad(x, delta, eps)
    fd = np.zeros_like(x)
    hstep = 1e-6
    for i in np.ndindex(x.shape):
        xp = x.copy(); xp[i] += hstep
        xm = x.copy(); xm[i] -= hstep
        fd[i] = (orc.awtv(xp, delta, eps, wref=x) - orc.awtv(xm, delta, eps, wref=x)) / (2 * hstep)
    assert _rel(g, fd) < 1e-7


def test_tv_steepest_descent_step_reduces_tv(orc):
    rng = np.random.Generator(np.random.PCG64(51))
    x = rng.random((8, 8, 8))
    g = orc.awtv_grad(x, eps=1e-8)
    x1 = x - 1e-3 * g / np.linalg.norm(g)
    assert orc.awtv(x1, eps=1e-8) < orc.awtv(x, eps=1e-8)


@pytest.mark.parametrize("blocksize", [1, 4])
def test_asd_pocs_without_tv_steps_is_os_sart_with_decaying_step(orc, blocksize):
    """With no TV steps (ng = 0) ASD-POCS is OS-SART whose step shrinks by
    lam_red every pass."""
    geo = _EMGEO
    ang = synth.circular_angles(8)
    rng = np.random.Generator(np.random.PCG64(52))
    b = orc.forward(geo, ang, rng.random(geo.nVoxel), "interp")
    got = orc.asd_pocs(geo, ang, b, 3, blocksize=blocksize, ng=0, lam=0.9, lam_red=0.8, kind="interp")
    x = None
    lam = 0.9
    for _ in range(3):
        x = orc.os_sart(geo, ang, b, 1, blocksize, lam=lam, nonneg=True, kind="interp", x0=x)
        lam *= 0.8
    assert _rel(got, x) < 1e-13


def test_asd_pocs_beats_os_sart_on_sparse_piecewise_constant(orc):
    """On a piecewise-constant phantom from 6 views, the TV steps lower the
    error of the same number of data passes."""
    geo = Geometry(DSD=60.0, DSO=40.0, nVoxel=(10, 10, 10), dVoxel=(1.0, 1.0, 1.0), nDetector=(12, 12),
                   dDetector=(1.4, 1.4))
    ang = synth.circular_angles(6)
    xt = np.zeros(geo.nVoxel)
    xt[2:8, 3:7, 2:8] = 1.0
    xt[4:6, 4:6, 4:6] = 2.0
    b = orc.forward(geo, ang, xt, "interp")
    xs = orc.os_sart(geo, ang, b, 10, 1, kind="interp")
    xa = orc.asd_pocs(geo, ang, b, 10, blocksize=1, kind="interp")
    assert np.linalg.norm(xa - xt) < np.linalg.norm(xs - xt)


# ------------------------------------------------------------------ PSNR
def test_psnr_closed_form():
    import oracle
    rng = np.random.Generator(np.random.PCG64(45))
    g = rng.random((4, 5, 6))
    g[0, 0, 0] = 0.0
    g[1, 1, 1] = 2.0
    x = g + 0.01
    assert abs(oracle.psnr(x, g) - 20 * math.log10(2.0 / 0.01)) < 1e-10


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_gradient_voxels_matches_dense_normal_equations(orc, kind):
    """The per-voxel gradient 2 (A^T (A x - y))_j against 2 M^T (M x - y)
    with the explicit matrix."""
    geo = TINY
    ang = _angles(4, 51)
    M = orc.dense_matrix(geo, ang, kind)
    rng = np.random.Generator(np.random.PCG64(52))
    x = rng.random(geo.nVoxel)
    y = rng.random((len(ang),) + geo.nDetector)
    want = 2.0 * M.T @ (M @ x.ravel() - y.ravel())
    sel = rng.integers(0, geo.n_vox, 40)
    iz, iy, ix = np.unravel_index(sel, geo.nVoxel)
    got = orc.gradient_voxels(geo, ang, x, y, iz, iy, ix, kind)
    assert np.allclose(got, want[sel], rtol=1e-11, atol=1e-11 * np.abs(want).max())


def test_bfdk_voxels_equals_full_backprojector(orc):
    geo = TINY_ANISO
    ang = _angles(6, 53)
    q = np.random.Generator(np.random.PCG64(54)).random((6,) + geo.nDetector)
    full = orc.bfdk(geo, ang, q)
    sel = np.arange(0, geo.n_vox, 7)
    iz, iy, ix = np.unravel_index(sel, geo.nVoxel)
    assert np.array_equal(orc.bfdk_voxels(geo, ang, q, iz, iy, ix), full.ravel()[sel])


# ------------------------------------------------------------ PnP-CGLS
def _pnp_setup():
    from synth import Geometry
    geo = Geometry(DSD=400.0, DSO=250.0, nVoxel=(16, 16, 16), dVoxel=(1.0, 1.0, 1.0), nDetector=(24, 24),
                   dDetector=(1.5, 1.5))
    ang = synth.circular_angles(12)
    x_gt = synth.voxelize(geo, synth.random_ellipsoids(geo, 5), dtype=np.float64)
    return geo, ang, x_gt


def test_pnp_cgls_rejected_denoiser_is_plain_cgls(orc):
    geo, ang, x_gt = _pnp_setup()
    b = orc.forward(geo, ang, x_gt, "interp")
    x0, h0 = orc.cgls(geo, ang, b, 12, kind="interp")
    bad = lambda x: x + 100.0                      # residual explodes: always rejected
    x1, h1 = orc.pnp_cgls(geo, ang, b, 12, bad, every=4, kind="interp")
    assert h1["accepted"] == [False, False, False] and min(h1["ratios"]) > 10
    assert np.array_equal(x0, x1)
    assert np.allclose(h1["resid"], h0["resid"], rtol=0, atol=0)


def test_pnp_cgls_exact_denoiser_reaches_ground_truth(orc):
    """b = A x_gt exactly; a denoiser returning x_gt has residual 0, is
    accepted, and the restarted CGLS stays there (gamma = 0)."""
    geo, ang, x_gt = _pnp_setup()
    b = orc.forward(geo, ang, x_gt, "siddon")
    x, h = orc.pnp_cgls(geo, ang, b, 10, lambda x: x_gt, every=5, kind="siddon", x_gt=x_gt)
    assert h["accepted"][0] and h["ratios"][0] < 1e-12
    assert np.array_equal(x, x_gt) and h["psnr"][-1] == np.inf
    assert h["resid"][4] < 1e-9 and h["resid"][-1] < 1e-9


def test_pnp_cgls_identity_denoiser_restarts_cgls(orc):
    """The identity is always accepted (ratio 1 up to the recurrence's
    drift) and restarts CGLS, which is then CGLS started from x_5."""
    geo, ang, x_gt = _pnp_setup()
    b = orc.forward(geo, ang, x_gt, "interp")
    x, h = orc.pnp_cgls(geo, ang, b, 9, lambda x: x, every=5, kind="interp")
    assert h["accepted"] == [True] and abs(h["ratios"][0] - 1.0) < 1e-9
    x5, _ = orc.cgls(geo, ang, b, 5, kind="interp")
    # four more CGLS steps from x5 with r = b - A x5
    r = b - orc.forward(geo, ang, x5, "interp")
    s = orc.backward(geo, ang, r, "interp")
    p, gam, xx = s.copy(), float(np.vdot(s, s)), x5.copy()
    for _ in range(4):
        q = orc.forward(geo, ang, p, "interp")
        al = gam / float(np.vdot(q, q))
        xx, r = xx + al * p, r - al * q
        s = orc.backward(geo, ang, r, "interp")
        g2 = float(np.vdot(s, s))
        p, gam = s + (g2 / gam) * p, g2
    assert np.max(np.abs(x - xx)) < 1e-10 * np.max(np.abs(xx))


# ------------------------------------------- ASD-POCS step-size control
_POCS_GEO = Geometry(DSD=60.0, DSO=40.0, nVoxel=(8, 8, 8), dVoxel=(1.0, 1.0, 1.0), nDetector=(10, 10),
                     dDetector=(1.4, 1.4))
_POCS = dict(blocksize=2, kind="interp", lam=1.0, lam_red=0.9, alpha=0.02, alpha_red=0.7, ng=5, rmax=0.5,
             eps_data=3.0, delta=math.inf, eps_tv=1e-8)


def _check_asd_pocs_trace(orc, asd_pocs, niter=8):
    """Re-derives ASD-POCS (Sidky and Pan's steps, the paper's POCS class
    of section 2.2 with its OS form of section 2.2.2) from pinned pieces --
    one OS-SART pass (oracle.os_sart) and the TV gradient (oracle.awtv_grad)
    -- and checks every iteration's dp, dd, dg, TV step length and data step
    against the trace of `asd_pocs`, then the image.  The step length starts
    at alpha dp and is multiplied by alpha_red after an iteration whose TV
    change dg exceeds rmax dp while the data residual dd is above eps_data;
    lam shrinks by lam_red every iteration.  Returns the decisions taken."""
    geo, p = _POCS_GEO, _POCS
    ang = synth.circular_angles(6)
    xt = np.zeros(geo.nVoxel)
    xt[2:6, 2:7, 1:6] = 1.0
    xt[3:5, 3:5, 3:5] = 2.0
    b = orc.forward(geo, ang, xt, "interp")
    trace = []
    got = asd_pocs(geo, ang, b, niter, trace=trace, **p)
    assert len(trace) == niter
    x = np.zeros(geo.nVoxel)
    lam, dtvg, events = p["lam"], None, []
    for k in range(niter):
        x_prev = x
        x = orc.os_sart(geo, ang, b, 1, p["blocksize"], lam=lam, nonneg=True, kind="interp", x0=x)
        dd = float(np.linalg.norm(orc.forward(geo, ang, x, "interp") - b))
        dp = float(np.linalg.norm(x - x_prev))
        if dtvg is None:
            dtvg = p["alpha"] * dp
        x_tv = x
        for _ in range(p["ng"]):
            g = orc.awtv_grad(x, p["delta"], p["eps_tv"])
            x = x - dtvg * g / np.linalg.norm(g)
        dg = float(np.linalg.norm(x - x_tv))
        t = trace[k]
        for name, want in (("dp", dp), ("dd", dd), ("dg", dg), ("dtvg", dtvg), ("lam", lam)):
            assert abs(t[name] - want) <= 1e-10 * abs(want), (k, name, t[name], want)
        over, noisy = dg > p["rmax"] * dp, dd > p["eps_data"]
        events.append((over, noisy))
        if over and noisy:
            dtvg *= p["alpha_red"]
        lam *= p["lam_red"]
    assert _rel(got, x) < 1e-10
    return events


def test_asd_pocs_step_size_trace(orc):
    events = _check_asd_pocs_trace(orc, orc.asd_pocs)
    # the rule fires, holds below rmax, and holds above rmax once the data
    # residual is within eps_data: every branch is taken before the last
    # iteration, so a wrong decision shows in a later step length
    assert (True, True) in events[:-1]
    assert any(not over for over, _ in events[:-1])
    assert (True, False) in events[:-1]


@pytest.mark.parametrize("old,new", [
    ("if dg > rmax * dp and dd > eps_data:", "if dg < rmax * dp and dd > eps_data:"),
    ("if dg > rmax * dp and dd > eps_data:", "if dg > rmax * dp:"),
    ("if dg > rmax * dp and dd > eps_data:", "if dg > rmax * dg and dd > eps_data:"),
    ("dtvg = alpha * dp", "dtvg = alpha * dd"),
    ("        lam *= lam_red\n", "        lam *= 1.0\n"),
    ("dtvg *= alpha_red", "dtvg *= lam_red"),
], ids=["inverted", "no-data-tolerance", "dg-vs-dg", "start-from-dd", "no-lam-decay", "wrong-factor"])
def test_asd_pocs_trace_pin_catches_planted_mistakes(orc, old, new):
    from _mutants import py_oracle_mutant
    mutant = py_oracle_mutant(orc.asd_pocs, old, new)
    with pytest.raises(AssertionError):
        _check_asd_pocs_trace(orc, mutant)
