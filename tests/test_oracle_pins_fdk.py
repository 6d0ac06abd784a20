"""Pins of the oracle's FDK weights and ramp that the 1 m-source tests cannot
see: a wide cone (DSO 150 mm, DSD 300 mm) where the cosine pre-weight falls
to 0.86 at the detector corner, and the parallel-beam limit.

FDK (the paper's direct method, section 2.1; Feldkamp, Davis and Kress
1984) is exact for objects that do not vary along the rotation axis: the
cosine weight DSD / sqrt(DSD^2 + u^2 + v^2) is the fan-beam weight times
the cosine of the ray's tilt out of the mid-plane, which cancels the longer
oblique path through a z-invariant object.  So a long uniform cylinder
reconstructs to its density on every slice, mid-plane or not.  Each planted
mistake below (weight dropped, DSO in place of DSD, v^2 left out, the 1/2
of the full-orbit redundancy dropped) breaks that on some slice.
"""
import math

import numpy as np
import pytest

import synth
from synth import Ellipsoid, Geometry

from _mutants import c_oracle_mutant

WIDE = Geometry(DSD=300.0, DSO=150.0, nVoxel=(96, 128, 128), dVoxel=(1.0, 1.0, 1.0), nDetector=(176, 160),
                dDetector=(1.5, 1.5))
WIDE_N = 180
R_CYL = 50.0


def _cylinder(r, cx=0.0, cy=0.0):
    return Ellipsoid((cx, cy, 0.0), (r, r, 1e5), ((1, 0, 0), (0, 1, 0), (0, 0, 1)), 1.0)


def _wide_fan_slices(orc, pa):
    """Interior (r < 0.8 R) of the mid-plane slice and of slices 40 mm
    above and below it, from the full FDK (filter, then B_FDK)."""
    ang = synth.circular_angles(WIDE_N)
    q = orc.fdk_filter(WIDE, pa, WIDE_N)
    c = np.arange(128) + 0.5 - 64
    Y, X = np.meshgrid(c, c, indexing="ij")
    iy, ix = np.nonzero(Y ** 2 + X ** 2 < (0.8 * R_CYL) ** 2)
    out = {}
    for iz in (47, 48, 7, 88):       # z = -0.5, +0.5, -40.5, +40.5 mm
        out[iz] = orc.bfdk_voxels(WIDE, ang, q, np.full(len(iy), iz), iy, ix)
    return out


def _check_unit_density(slices):
    for iz, f in slices.items():
        assert abs(f.mean() - 1.0) < 5e-3, (iz, f.mean())
        assert np.max(np.abs(f - 1.0)) < 1e-2, (iz, np.max(np.abs(f - 1.0)))


@pytest.fixture(scope="module")
def wide_projections(orc):
    return orc.analytic_projections(WIDE, synth.circular_angles(WIDE_N), [_cylinder(R_CYL)])


def test_wide_fan_geometry_exercises_the_cosine_weight():
    """The detector corner sees DSD / sqrt(DSD^2 + u^2 + v^2) = 0.86, and
    the cylinder's shadow reaches u = 106 mm (weight 0.94 in the mid-row);
    the voxels 40.5 mm off the mid-plane are seen in every view."""
    nv, nu = WIDE.nDetector
    u, v = nu / 2 * WIDE.dDetector[1], nv / 2 * WIDE.dDetector[0]
    assert WIDE.DSD / math.sqrt(WIDE.DSD ** 2 + u * u + v * v) < 0.87
    shadow = WIDE.DSD * R_CYL / math.sqrt(WIDE.DSO ** 2 - R_CYL ** 2)
    assert 100.0 < shadow < u
    # highest voxel row used, at the ball's nearest approach to the source
    assert WIDE.DSD * 41.0 / (WIDE.DSO - 0.8 * R_CYL) < v


def test_fdk_wide_fan_cylinder_every_slice(orc, wide_projections):
    _check_unit_density(_wide_fan_slices(orc, wide_projections))


_W = "double w = g->DSD / sqrt(g->DSD * g->DSD + u * u + v * v);"


@pytest.mark.parametrize("new", [
    "double w = 1.0;",                                                   # cosine weight dropped
    "double w = g->DSO / sqrt(g->DSO * g->DSO + u * u + v * v);",        # DSO in place of DSD
    "double w = g->DSD / sqrt(g->DSD * g->DSD + u * u);",                # v^2 left out
], ids=["weight-dropped", "dso-for-dsd", "no-v2"])
def test_wide_fan_pin_catches_planted_weight_mistakes(orc, wide_projections, tmp_path, new):
    with c_oracle_mutant(tmp_path, _W, new):
        slices = _wide_fan_slices(orc, wide_projections)
    with pytest.raises(AssertionError):
        _check_unit_density(slices)


def test_wide_fan_pin_catches_dropped_redundancy_half(orc, wide_projections, tmp_path):
    with c_oracle_mutant(tmp_path, "const double scale = wang ? dtheta : 0.5 * dtheta;",
                         "const double scale = dtheta;"):
        slices = _wide_fan_slices(orc, wide_projections)
    with pytest.raises(AssertionError):
        _check_unit_density(slices)


def _parallel_fbp(ang, nu, tau, R, cx, cy, n):
    """Textbook parallel-beam filtered backprojection of a unit disc on an
    n x n grid of 1 mm pixels (Kak and Slaney, ch. 3): the disc's Radon
    transform 2 sqrt(R^2 - (s - s_c)^2) sampled at s_i = (i + 1/2 - nu/2) tau,
    convolved with the spatial Ram-Lak kernel (numpy's linear convolution),
    linearly interpolated at s = -x sin(t) + y cos(t), summed with weight
    pi / N over the N views of the full orbit."""
    s = (np.arange(nu) + 0.5 - nu / 2) * tau
    k = np.arange(-(nu - 1), nu).astype(np.float64)
    h = np.zeros_like(k)
    h[k == 0] = 1.0 / (4.0 * tau * tau)
    odd = np.abs(k) % 2 == 1
    h[odd] = -1.0 / (k[odd] ** 2 * math.pi ** 2 * tau * tau)
    c = np.arange(n) + 0.5 - n / 2
    X, Y = np.meshgrid(c, c, indexing="xy")
    f = np.zeros((n, n))
    for t in ang:
        sc = -cx * math.sin(t) + cy * math.cos(t)
        p = 2.0 * np.sqrt(np.maximum(R * R - (s - sc) ** 2, 0.0))
        q = tau * np.convolve(p, h, mode="full")[nu - 1:2 * nu - 1]
        f += np.interp(-X * math.sin(t) + Y * math.cos(t), s, q, left=0.0, right=0.0)
    return f * math.pi / len(ang), X, Y


def test_fdk_parallel_limit_equals_parallel_fbp(orc):
    """With the source 1 km away (DSO = 10^6 mm, DSD = 1.536 DSO) the
    oracle's FDK of an off-centre z-invariant disc equals the parallel-beam
    FBP of the same disc at every pixel of the central slices (the fan and
    cone angles are below 5e-5 rad), and reconstructs the unit density."""
    DSO, tau, nu, n = 1e6, 0.75, 128, 64
    geo = Geometry(DSD=1.536 * DSO, DSO=DSO, nVoxel=(4, n, n), dVoxel=(1.0, 1.0, 1.0), nDetector=(8, nu),
                   dDetector=(1.536, 1.536 * tau))
    ang = synth.circular_angles(256)
    R, cx, cy = 20.0, 5.0, -3.0
    f = orc.fdk(geo, ang, orc.analytic_projections(geo, ang, [_cylinder(R, cx, cy)]))
    fp, X, Y = _parallel_fbp(ang, nu, tau, R, cx, cy, n)
    for iz in (1, 2):
        assert np.max(np.abs(f[iz] - fp)) < 2e-4
    inside = (X - cx) ** 2 + (Y - cy) ** 2 < (0.8 * R) ** 2
    assert abs(f[1][inside].mean() - 1.0) < 1e-3
    outside = (X - cx) ** 2 + (Y - cy) ** 2 > (1.2 * R) ** 2
    assert abs(f[1][outside].mean()) < 1e-2
