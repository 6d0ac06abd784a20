"""The projectors' less common paths against the FP64 oracle, through the C
ABI (tolerance rel-L2 1e-4, as for every projector):

* views whose tiles straddle a diagonal of the orbit plane: a tile with a
  ray running as steep along another axis as along the tile's dominant one
  (to 1 %) walks its layers plane by plane in the Siddon forward, and the
  Siddon adjoint walks such rays' items plane by plane;
* a coarse detector (pixels several voxels wide), whose 16 x 16 ray bundles
  are wider than the forward kernels' LDS box can hold: the boxes are clipped
  to the capacity, so rays leave them and read global memory (Siddon: layer
  by layer outside the box; interpolated: the checked sample loop)."""
import numpy as np
import pytest

from synth import Geometry

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import synth  # noqa: E402

DIAG = Geometry(DSD=400.0, DSO=250.0, nVoxel=(36, 48, 44), dVoxel=(1.0, 1.0, 1.0), nDetector=(40, 72),
                dDetector=(1.2, 1.2), offOrigin=(0.3, -0.6, 0.2), offDetector=(0.4, -0.7))
# 4 mm pixels at a magnification of 1.6: one pixel spans about 5 voxels at the
# axis, a 16-pixel tile more than the whole 48-voxel cross-section
COARSE = Geometry(DSD=400.0, DSO=250.0, nVoxel=(40, 48, 48), dVoxel=(0.5, 0.5, 0.5), nDetector=(20, 24),
                  dDetector=(4.0, 4.0))


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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _diagonal_angles():
    q = np.pi / 4
    return np.array([q, q + 0.002, q - 0.003, 3 * q, 3 * q + 0.004, 5 * q - 0.001, 7 * q, 7 * q + 0.0015])


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_diagonal_views(P, orc, kind):
    ang = _diagonal_angles()
    # some rays of the central tiles run within 1 % of 45 degrees in the
    # orbit plane (the plane-by-plane case)
    S = np.array([DIAG.DSO * np.cos(ang[0]), DIAG.DSO * np.sin(ang[0])])
    d = -S
    assert abs(abs(d[0]) / abs(d[1]) - 1.0) < 0.01
    plan = P.Plan(DIAG, ang)
    x = synth.uniform_volume(DIAG, 31)
    y = synth.uniform_projections(DIAG, len(ang), 32)
    fx = _host(plan.forward(_dev(x), kind=kind))
    assert _rel(fx, orc.forward(DIAG, ang, x, kind)) < 1e-4
    bt = _host(plan.backproject(_dev(y), kind=kind))
    assert _rel(bt, orc.backward(DIAG, ang, y, kind)) < 1e-4
    # the pair stays matched: <A x, y> = <x, A^T y>
    lhs = float(np.dot(fx.astype(np.float64).ravel(), y.astype(np.float64).ravel()))
    rhs = float(np.dot(x.astype(np.float64).ravel(), bt.astype(np.float64).ravel()))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


@pytest.mark.parametrize("kind", ["siddon", "interp"])
def test_coarse_detector_overflows_the_box(P, orc, kind):
    rng = np.random.Generator(np.random.PCG64(33))
    ang = np.sort(rng.uniform(0, 2 * np.pi, 10))
    plan = P.Plan(COARSE, ang)
    x = synth.uniform_volume(COARSE, 34)
    y = synth.uniform_projections(COARSE, len(ang), 35)
    assert _rel(_host(plan.forward(_dev(x), kind=kind)), orc.forward(COARSE, ang, x, kind)) < 1e-4
    assert _rel(_host(plan.backproject(_dev(y), kind=kind)), orc.backward(COARSE, ang, y, kind)) < 1e-4
