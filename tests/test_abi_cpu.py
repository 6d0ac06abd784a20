"""Host-side checks of libctmi that need no GPU: the library loads, exports
every symbol its header declares, validates arguments before touching the
device, and computes the per-view geometry table consistently with the
oracle's ray geometry."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import synth
from synth import Geometry

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ctmi():
    import paper_2412_10129_amd as P
    return P


def _header_symbols():
    syms = set()
    for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        syms |= set(re.findall(r"\b(ctmi_[a-z0-9_]+)\s*\(", src))
    return sorted(syms)


def test_library_exports_every_declared_symbol(ctmi):
    lib = ctmi.library()
    syms = _header_symbols()
    assert len(syms) >= 18
    for s in syms:
        assert hasattr(lib, s), s
    from paper_2412_10129_amd import _lib
    assert set(syms) == set(_lib.EXPORTED)


def test_binding_argument_counts_match_headers():
    """Every ctypes signature has as many arguments as the C declaration."""
    from paper_2412_10129_amd import _lib
    for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        for name, params in re.findall(r"\b(ctmi_[a-z0-9_]+)\s*\(([^)]*)\)\s*;", src):
            params = params.strip()
            n = 0 if params in ("", "void") else params.count(",") + 1
            assert len(_lib._SIGS[name][1]) == n, (name, n, len(_lib._SIGS[name][1]))


def test_version_and_error_string(ctmi):
    lib = ctmi.library()
    assert b"gfx950" in lib.ctmi_version()
    assert isinstance(lib.ctmi_last_error(), bytes)


def _bad(geo, **kw):
    return geo.replace(**kw)


@pytest.mark.parametrize("change,exc", [
    (dict(DSO=10.0), ValueError),                   # source inside the volume
    (dict(DSD=1040.0), ValueError),                 # detector cuts the volume
    (dict(DSD=900.0), ValueError),                  # DSD < DSO
    (dict(nVoxel=(64, 0, 64)), ValueError),
    (dict(dVoxel=(1.0, -1.0, 1.0)), ValueError),
    (dict(dDetector=(1.6, float("nan"))), ValueError),
    (dict(accuracy=0.0), ValueError),
    (dict(offOrigin=(0.0, float("inf"), 0.0)), ValueError),
])
def test_geometry_validation(ctmi, change, exc):
    geo, ang = synth.workload("head64")
    with pytest.raises(exc):
        ctmi.geometry_check(_bad(geo, **change), ang)


def test_unsupported_features_are_reported(ctmi):
    geo, ang = synth.workload("head64")

    class G:
        pass

    g = G()
    for k in ("DSD", "DSO", "nVoxel", "dVoxel", "nDetector", "dDetector", "offOrigin", "offDetector", "accuracy"):
        setattr(g, k, getattr(geo, k))
    g.COR = 1.0
    with pytest.raises(NotImplementedError):
        ctmi.geometry_check(g, ang)
    g.COR = 0.0
    g.rotDetector = (0.0, 0.1, 0.0)
    with pytest.raises(NotImplementedError):
        ctmi.geometry_check(g, ang)


def test_bad_angles_and_sizes(ctmi):
    geo, ang = synth.workload("head64")
    bad = ang.copy()
    bad[3] = np.nan
    with pytest.raises(ValueError):
        ctmi.geometry_check(geo, bad)
    with pytest.raises(ValueError):
        ctmi.geometry_check(geo, ang[:0])
    big = geo.replace(nVoxel=(2048, 2048, 1024), dVoxel=(0.01, 0.01, 0.01))
    from paper_2412_10129_amd import CtmiError
    with pytest.raises(CtmiError):
        ctmi.geometry_check(big, ang)
    # detectors: nu <= 4096, and fewer than 2^28 pixels (int32 footprint counts)
    with pytest.raises(CtmiError, match="nu <= 4096"):
        ctmi.geometry_check(geo.replace(nDetector=(64, 4097)), ang)
    with pytest.raises(CtmiError, match="2\\^28"):
        ctmi.geometry_check(geo.replace(nDetector=(65536, 4096), dDetector=(0.001, 0.001)), ang)
    ctmi.geometry_check(geo.replace(nDetector=(65535, 4096), dDetector=(0.001, 0.001)), ang)


def test_null_arguments_fail_before_any_device_call(ctmi):
    lib = ctmi.library()
    assert lib.ctmi_forward(None, 0, None, None, 0, 1, None) == -1
    assert b"plan is NULL" in lib.ctmi_last_error()
    assert lib.ctmi_plan_create(None, None, 1, ctypes.byref(ctypes.c_void_p())) == -1
    assert lib.ctmi_dot(None, None, 10, None, None, 0, None) == -1
    assert lib.ctmi_plan_destroy(None) == 0
    assert lib.ctmi_axpby(-1, 1.0, None, 1.0, None, None) == -1


def test_view_table_matches_oracle_ray_geometry(ctmi, orc):
    """Source and pixel positions of the device table (voxel-cell
    coordinates) map back to the oracle's world-frame ray end points, and the
    projection matrix rows send a voxel centre to the pixel where the line
    source-voxel meets the detector."""
    geo = Geometry(DSD=300.0, DSO=200.0, nVoxel=(6, 8, 10), dVoxel=(2.0, 1.5, 1.0), nDetector=(40, 50),
                   dDetector=(1.5, 1.3), offOrigin=(1.0, -2.0, 3.0), offDetector=(0.7, -0.9))
    ang = np.array([0.0, 0.7, 2.9, 4.4])
    t = ctmi.view_table(geo, ang).astype(np.float64)
    nz, ny, nx = geo.nVoxel
    h = np.array(geo.dVoxel[::-1])
    lo = np.array(geo.offOrigin[::-1]) - np.array([nx, ny, nz]) * h / 2
    for k, th in enumerate(ang):
        for iv, iu in [(0, 0), (3, 17), (39, 49)]:
            S, P = orc.ray_endpoints(geo, th, iv, iu)
            St = lo + t[k, 0:3] * h
            Pt = lo + (t[k, 3:6] + iu * t[k, 6:9] + iv * t[k, 9:12]) * h
            assert np.allclose(St, S, atol=2e-4 * geo.DSO)
            assert np.allclose(Pt, P, atol=2e-4 * geo.DSD)
        _, P00 = orc.ray_endpoints(geo, th, 0.0, 0.0)
        _, P01 = orc.ray_endpoints(geo, th, 0.0, 1.0)
        _, P10 = orc.ray_endpoints(geo, th, 1.0, 0.0)
        S, _ = orc.ray_endpoints(geo, th, 0.0, 0.0)
        for (iz, iy, ix) in [(0, 0, 0), (5, 7, 9), (2, 3, 4)]:
            X = lo + (np.array([ix, iy, iz]) + 0.5) * h
            A = np.stack([X - S, -(P01 - P00), -(P10 - P00)], 1)
            _, fu, fv = np.linalg.solve(A, P00 - S)
            c = np.array([ix, iy, iz, 1.0])
            W = t[k, 20:24] @ c
            assert abs(t[k, 12:16] @ c / W - fu) < 1e-3
            assert abs(t[k, 16:20] @ c / W - fv) < 1e-3
            U = geo.DSO - (X[0] * np.cos(th) + X[1] * np.sin(th))
            assert abs(W - U / geo.DSO) < 1e-6
