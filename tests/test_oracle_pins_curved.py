"""Pins of the oracle's curved-detector flattening (the paper's curved
detectors, section 2.4: a curved detector is handled by a flattening
transformation onto a flat one).

The flattening carries each flat pixel's ray over to the curved detector,
so the pins use what fixes a ray and its line integral independently of the
resampling: closed-form line integrals of smooth Gaussian blobs to the
curved pixel centres, flattened, must converge to the closed-form integrals
to the flat pixel centres at second order in the curved pitch (smooth
projections, so bilinear resampling is second order); the arc of radius
DSD keeps every pixel of a row at the same distance from the source; a huge
radius is the flat detector.  Planted mistakes in the transformation fail
the convergence pin."""
import math

import numpy as np
import pytest

import synth
from _mutants import py_oracle_mutant
from synth import CurvedDetector, Geometry

# wide fan: the flat detector spans +-17.7 degrees, so the arc and the flat
# plane differ by 5 % in depth at the edges
GEO = Geometry(DSD=600.0, DSO=400.0, nVoxel=(64, 64, 64), dVoxel=(1.0, 1.0, 1.0), nDetector=(96, 192),
               dDetector=(2.0, 2.0))
ANG = np.array([0.3, 1.9, 3.4, 5.0])


def _curved(R, pitch):
    """A curved detector covering the flat one's rays with margin, its pixel
    grid shifted by a fixed fraction of a pixel so that no resolution lines
    its centres up with the flat ones."""
    half_u = R * 0.40            # arc length beyond the widest ray
    half_v = 0.5 * GEO.nDetector[0] * GEO.dDetector[0] + 4.0
    return CurvedDetector(nDetector=(2 * int(math.ceil(half_v / pitch)), 2 * int(math.ceil(half_u / pitch))),
                          dDetector=(pitch, pitch), radius=R, offDetector=(0.37 * pitch, 0.61 * pitch))


# Gaussian blobs rho exp(-|x - c|^2 / (2 sigma^2)): the integral along a line
# at distance d from c is rho sigma sqrt(2 pi) exp(-d^2 / (2 sigma^2))
# (spread over the fan and the detector height, so that the depth and height
# rescaling of the arc matter; the line integrals need no voxel grid)
BLOBS = [((0.0, 0.0, 0.0), 14.0, 1.0), ((60.0, -40.0, 35.0), 12.0, 0.6), ((-70.0, 50.0, -40.0), 15.0, 0.8),
         ((40.0, 80.0, 60.0), 10.0, 0.5)]


def _blob_integrals(S, P):
    d = P - S
    dh = d / np.linalg.norm(d, axis=-1, keepdims=True)
    out = np.zeros(P.shape[:-1])
    for c, sig, rho in BLOBS:
        w = np.asarray(c) - S
        perp = w - np.sum(w * dh, -1, keepdims=True) * dh
        out += rho * sig * math.sqrt(2 * math.pi) * np.exp(-np.sum(perp * perp, -1) / (2 * sig * sig))
    return out


def _analytic_curved(orc, ells, cd):
    out = []
    for th in ANG:
        S = GEO.DSO * np.array([math.cos(th), math.sin(th), 0.0])
        P = orc.curved_pixel_centres(GEO, th, cd)
        out.append(_blob_integrals(np.broadcast_to(S, P.shape), P))
    return np.stack(out)


@pytest.fixture(scope="module")
def ells():
    return BLOBS


@pytest.fixture(scope="module")
def flat_truth(orc):
    out = []
    nv, nu = GEO.nDetector
    for th in ANG:
        P = np.zeros((nv, nu, 3))
        for iv in range(nv):
            for iu in range(nu):
                S, P[iv, iu] = orc.ray_endpoints(GEO, th, iv, iu)
        out.append(_blob_integrals(np.broadcast_to(S, P.shape), P))
    return np.stack(out)


def _err(orc, ells, flat_truth, R, pitch, fn=None):
    cd = _curved(R, pitch)
    fl = (fn or orc.flatten_curved)(GEO, cd, _analytic_curved(orc, ells, cd))
    return float(np.linalg.norm(fl - flat_truth) / np.linalg.norm(flat_truth))


def test_arc_of_radius_dsd_is_equidistant(orc):
    cd = CurvedDetector(nDetector=(9, 31), dDetector=(1.5, 3.0), radius=GEO.DSD, offDetector=(0.7, 2.0))
    for th in ANG:
        S = GEO.DSO * np.array([math.cos(th), math.sin(th), 0.0])
        P = orc.curved_pixel_centres(GEO, th, cd)
        horiz = np.hypot(P[..., 0] - S[0], P[..., 1] - S[1])
        assert np.allclose(horiz, GEO.DSD, rtol=0, atol=1e-9)
        # neighbouring columns subtend du / R at the source
        d = P[0, :, :2] - S[:2]
        ang = np.arctan2(d[:, 1], d[:, 0])
        assert np.allclose(np.abs(np.diff(np.unwrap(ang))), 3.0 / GEO.DSD, rtol=0, atol=1e-12)
        # the centre column (arc length 0 at offset 0) sits on the flat detector's centre line
        assert np.allclose(P[:, :, 2], (np.arange(9) + 0.5 - 4.5)[:, None] * 1.5 + 0.7)


def test_huge_radius_is_the_flat_detector(orc):
    cd = CurvedDetector(nDetector=GEO.nDetector, dDetector=GEO.dDetector, radius=1e9)
    for th in ANG[:2]:
        P = orc.curved_pixel_centres(GEO, th, cd)
        for iv, iu in ((0, 0), (40, 100), (95, 191)):
            _, Pf = orc.ray_endpoints(GEO, th, iv, iu)
            assert np.allclose(P[iv, iu], Pf, rtol=0, atol=1e-4)
    q = synth.uniform_projections(GEO, 3, 1).astype(np.float64)
    assert np.max(np.abs(orc.flatten_curved(GEO, cd, q) - q)) < 1e-5


def test_centre_column_carries_over_exactly(orc):
    """A flat pixel whose ray runs through a curved pixel centre takes that
    pixel's value: with an odd column count and no offsets the centre
    column maps to arc length 0, and with R = DSD its heights are unscaled."""
    geo = GEO.replace(nDetector=(96, 191))
    cd = CurvedDetector(nDetector=(96, 201), dDetector=GEO.dDetector, radius=GEO.DSD)
    q = synth.uniform_projections(geo.replace(nDetector=cd.nDetector), 2, 2).astype(np.float64)
    fl = orc.flatten_curved(geo, cd, q)
    assert np.array_equal(fl[:, :, 95], q[:, :, 100])


@pytest.mark.parametrize("R", [600.0, 900.0])
def test_flattened_closed_form_converges_at_second_order(orc, ells, flat_truth, R):
    e1 = _err(orc, ells, flat_truth, R, 2.0)
    e2 = _err(orc, ells, flat_truth, R, 1.0)
    e4 = _err(orc, ells, flat_truth, R, 0.5)
    assert e1 < 2e-2 and e4 < 2e-3, (e1, e2, e4)
    assert e1 / e2 > 2.5 and e2 / e4 > 2.5, (e1, e2, e4)


MUTANTS = [
    # heights not rescaled to the cylinder
    ("vc = t[None, :] * vf[:, None]", "vc = np.ones_like(t)[None, :] * vf[:, None]", (600.0, 900.0)),
    # arc length taken as the flat coordinate
    ("s = R * np.arctan2(t * uf, t * DSD - DSD + R)", "s = uf * 1.0", (600.0, 900.0)),
    # the arc's angle measured at the source instead of the axis (the same
    # thing when the axis is the source, R = DSD)
    ("s = R * np.arctan2(t * uf, t * DSD - DSD + R)", "s = R * np.arctan2(uf, DSD)", (900.0,)),
    # the root behind the source
    ("t = (-b + np.sqrt(b * b - 4.0 * a * c)) / (2.0 * a)", "t = (-b - np.sqrt(b * b - 4.0 * a * c)) / (2.0 * a)",
     (600.0, 900.0)),
]


@pytest.mark.parametrize("old,new,R", [(o, n, R) for o, n, Rs in MUTANTS for R in Rs])
def test_convergence_pin_catches_planted_mistakes(orc, ells, flat_truth, old, new, R):
    bad = py_oracle_mutant(orc.flatten_curved, old, new)
    e_ok = _err(orc, ells, flat_truth, R, 0.5)
    e_bad = _err(orc, ells, flat_truth, R, 0.5, fn=bad)
    assert e_bad > 10 * e_ok, (e_ok, e_bad)
