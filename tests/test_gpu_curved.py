"""GPU parity of the curved-detector flattening (section 2.4: curved
detectors are taken in through a flattening transformation) against the
FP64 oracle, through the C ABI, and FDK from curved-detector data.

Tolerance: rel-L2 1e-5 for the resampling itself (FP64 coordinates, FP32
weights and values) and 1e-4 for FDK after it (the parity bar of A and
A^T)."""
import math

import numpy as np
import pytest

import synth
from synth import CurvedDetector, Geometry

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GEO = Geometry(DSD=600.0, DSO=400.0, nVoxel=(40, 48, 44), dVoxel=(1.0, 1.0, 1.0), nDetector=(70, 150),
               dDetector=(1.3, 1.1), offDetector=(0.9, -2.3))


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_10129_amd as P
    return P


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("cd", [
    CurvedDetector(nDetector=(75, 161), dDetector=(1.25, 1.05), radius=600.0, offDetector=(0.4, 1.7)),
    CurvedDetector(nDetector=(64, 129), dDetector=(1.4, 1.3), radius=900.0, offDetector=(-0.3, 0.0)),
    # narrower than the flat detector: the outer flat columns fall outside (zeros)
    CurvedDetector(nDetector=(50, 97), dDetector=(1.1, 1.2), radius=350.0),
    CurvedDetector(nDetector=(70, 150), dDetector=(1.3, 1.1), radius=1e9, offDetector=(0.9, -2.3)),
])
def test_flatten_matches_oracle(P, orc, cd):
    ang = np.linspace(0.0, 2 * math.pi, 7, endpoint=False)
    q = synth.uniform_projections(GEO.replace(nDetector=cd.nDetector), len(ang), 3)
    plan = P.Plan(GEO, ang)
    got = plan.flatten_curved(torch.from_numpy(q).cuda(), cd)
    torch.cuda.synchronize()
    want = orc.flatten_curved(GEO, cd, q)
    got = got.cpu().numpy()
    assert _rel(got, want) < 1e-5, _rel(got, want)
    assert np.array_equal(got == 0, want == 0) or cd.radius != 350.0
    # a view sub-range flattens the same views
    part = plan.flatten_curved(torch.from_numpy(q[2:5].copy()).cuda(), cd, view0=2, nviews=3)
    torch.cuda.synchronize()
    assert np.array_equal(part.cpu().numpy(), got[2:5])


def test_flatten_argument_errors(P):
    plan = P.Plan(GEO, np.zeros(2))
    q = torch.zeros((2, 10, 20), device="cuda")
    for bad in (CurvedDetector((10, 20), (1.0, 1.0), radius=299.0), CurvedDetector((10, 20), (1.0, 0.0), radius=600.0),
                CurvedDetector((10, 20), (1.0, 1.0), radius=float("inf"))):
        with pytest.raises(ValueError):
            plan.flatten_curved(q, bad)
    views = synth.views(GEO, np.zeros(2))
    gplan = P.Plan(GEO, views)
    with pytest.raises(NotImplementedError):
        gplan.flatten_curved(q, CurvedDetector((10, 20), (1.0, 1.0), radius=600.0))


def test_fdk_from_curved_detector_data(P, orc):
    """Closed-form projections of the head phantom on an equidistant arc
    (R = DSD), flattened and reconstructed by FDK on the GPU, against the
    same chain in the oracle."""
    geo = Geometry(DSD=600.0, DSO=400.0, nVoxel=(48, 48, 48), dVoxel=(1.0, 1.0, 1.0), nDetector=(80, 96),
                   dDetector=(1.2, 1.2))
    ang = synth.circular_angles(48)
    cd = CurvedDetector(nDetector=(80, 101), dDetector=(1.2, 1.2), radius=geo.DSD)
    ells = synth.head_phantom(geo, 1)
    q = []
    for th in ang:
        S = geo.DSO * np.array([math.cos(th), math.sin(th), 0.0])
        Pc = orc.curved_pixel_centres(geo, th, cd)
        q.append(orc.ellipsoid_line_integrals(ells, np.broadcast_to(S, Pc.shape), Pc))
    q = np.stack(q).astype(np.float32)
    plan = P.Plan(geo, ang)
    flat = plan.flatten_curved(torch.from_numpy(q).cuda(), cd)
    rec = P.fdk(plan, flat)
    torch.cuda.synchronize()
    want = orc.fdk(geo, ang, orc.flatten_curved(geo, cd, q.astype(np.float64)))
    assert _rel(rec.cpu().numpy(), want) < 1e-4
