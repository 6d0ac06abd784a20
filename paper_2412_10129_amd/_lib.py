"""ctypes binding of libctmi.so: argument marshalling only.

Every computation happens in the HIP library.  If the library is missing the
import fails loudly; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; CTMI_LIB names another build of the same library (for
# instance one compiled with other tile or slab sizes)
LIB_PATH = os.environ.get("CTMI_LIB") or os.path.join(HERE, "libctmi.so")

CTMI_OK, CTMI_EINVAL, CTMI_EUNSUPPORTED, CTMI_EOVERFLOW, CTMI_EWORKSPACE, CTMI_EHIP = 0, -1, -2, -3, -4, -5
CTMI_SIDDON, CTMI_INTERP = 0, 1
CTMI_BP_SIDDON, CTMI_BP_INTERP, CTMI_BP_FDK = 0, 1, 2
(CTMI_OP_FORWARD_SIDDON, CTMI_OP_FORWARD_INTERP, CTMI_OP_BACKPROJECT_SIDDON, CTMI_OP_BACKPROJECT_INTERP,
 CTMI_OP_BACKPROJECT_FDK, CTMI_OP_FDK_FILTER, CTMI_OP_FOV_SQ_ERR) = range(7)

c_i64, c_f, c_d, c_p, c_int = ctypes.c_int64, ctypes.c_float, ctypes.c_double, ctypes.c_void_p, ctypes.c_int


class CtmiGeometry(ctypes.Structure):
    _fields_ = [("DSD", c_d), ("DSO", c_d), ("nVoxel", c_i64 * 3), ("dVoxel", c_d * 3), ("offOrigin", c_d * 3),
                ("nDetector", c_i64 * 2), ("dDetector", c_d * 2), ("offDetector", c_d * 2), ("COR", c_d),
                ("rotDetector", c_d * 3), ("accuracy", c_d)]


def geometry_struct(geo) -> CtmiGeometry:
    """From any object with the geometry-table attributes (DSD, DSO, nVoxel,
    dVoxel, nDetector, dDetector and optionally offOrigin, offDetector, COR,
    rotDetector, accuracy)."""
    g = CtmiGeometry()
    g.DSD = float(geo.DSD)
    g.DSO = float(geo.DSO)
    g.nVoxel = (c_i64 * 3)(*[int(v) for v in geo.nVoxel])
    g.dVoxel = (c_d * 3)(*[float(v) for v in geo.dVoxel])
    g.offOrigin = (c_d * 3)(*[float(v) for v in getattr(geo, "offOrigin", (0.0, 0.0, 0.0))])
    g.nDetector = (c_i64 * 2)(*[int(v) for v in geo.nDetector])
    g.dDetector = (c_d * 2)(*[float(v) for v in geo.dDetector])
    g.offDetector = (c_d * 2)(*[float(v) for v in getattr(geo, "offDetector", (0.0, 0.0))])
    g.COR = float(getattr(geo, "COR", 0.0))
    g.rotDetector = (c_d * 3)(*[float(v) for v in getattr(geo, "rotDetector", (0.0, 0.0, 0.0))])
    g.accuracy = float(getattr(geo, "accuracy", 0.5))
    return g


class CtmiView(ctypes.Structure):
    _fields_ = [("angles", c_d * 3), ("DSD", c_d), ("DSO", c_d), ("offOrigin", c_d * 3), ("offDetector", c_d * 2),
                ("COR", c_d), ("rotDetector", c_d * 3)]


class CtmiCurvedDetector(ctypes.Structure):
    _fields_ = [("nDetector", c_i64 * 2), ("dDetector", c_d * 2), ("offDetector", c_d * 2), ("radius", c_d)]


def curved_struct(cd) -> CtmiCurvedDetector:
    """From any object with nDetector (nv, nu), dDetector (dv, du), radius and
    optionally offDetector (v, u)."""
    c = CtmiCurvedDetector()
    c.nDetector = (c_i64 * 2)(*[int(v) for v in cd.nDetector])
    c.dDetector = (c_d * 2)(*[float(v) for v in cd.dDetector])
    c.offDetector = (c_d * 2)(*[float(v) for v in getattr(cd, "offDetector", (0.0, 0.0))])
    c.radius = float(cd.radius)
    return c


def view_structs(views):
    """ctmi_view records from a per-view description: any object with
    per-view arrays angles (n, 3) z1 y1 z2, DSO, DSD (n,), offOrigin (n, 3),
    offDetector (n, 2), COR (n,), rotDetector (n, 3)."""
    import numpy as np
    a = np.asarray(views.angles, dtype=np.float64).reshape(-1, 3)
    n = a.shape[0]
    col = lambda name, w: np.broadcast_to(np.asarray(getattr(views, name), dtype=np.float64), (n,) if w == 1 else (n, w))
    dso, dsd, cor = col("DSO", 1), col("DSD", 1), col("COR", 1)
    oo, od, rd = col("offOrigin", 3), col("offDetector", 2), col("rotDetector", 3)
    tab = (CtmiView * n)()
    for k in range(n):
        tab[k] = CtmiView((c_d * 3)(*a[k]), float(dsd[k]), float(dso[k]), (c_d * 3)(*oo[k]), (c_d * 2)(*od[k]),
                          float(cor[k]), (c_d * 3)(*rd[k]))
    return tab


_SIGS = {
    "ctmi_last_error": (ctypes.c_char_p, []),
    "ctmi_version": (ctypes.c_char_p, []),
    "ctmi_geometry_check": (c_int, [c_p, c_p, c_i64]),
    "ctmi_view_table": (c_int, [c_p, c_p, c_i64, c_p]),
    "ctmi_plan_create": (c_int, [c_p, c_p, c_i64, ctypes.POINTER(c_p)]),
    "ctmi_plan_create_views": (c_int, [c_p, c_p, c_i64, ctypes.POINTER(c_p)]),
    "ctmi_plan_destroy": (c_int, [c_p]),
    "ctmi_forward": (c_int, [c_p, c_int, c_p, c_p, c_i64, c_i64, c_p]),
    "ctmi_backproject": (c_int, [c_p, c_int, c_p, c_p, c_i64, c_i64, c_f, c_p, ctypes.c_size_t, c_p]),
    "ctmi_backproject_noalloc": (c_int, [c_p, c_int, c_p, c_p, c_i64, c_i64, c_f, c_p]),
    "ctmi_workspace_size": (c_int, [c_p, c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "ctmi_stream_check": (c_int, [c_p]),
    "ctmi_fdk_filter": (c_int, [c_p, c_int, c_p, c_p, c_i64, c_i64, c_p]),
    "ctmi_reduce_workspace_bytes": (ctypes.c_size_t, [c_i64]),
    "ctmi_dot": (c_int, [c_p, c_p, c_i64, c_p, c_p, ctypes.c_size_t, c_p]),
    "ctmi_axpby": (c_int, [c_i64, c_f, c_p, c_f, c_p, c_p]),
    "ctmi_cgls_xr": (c_int, [c_p, c_p, c_i64, c_p, c_p, c_i64, c_p, c_p, c_p, c_p, ctypes.c_size_t, c_p]),
    "ctmi_cgls_p": (c_int, [c_p, c_p, c_i64, c_p, c_p, c_p]),
    "ctmi_recip_or_zero": (c_int, [c_p, c_p, c_i64, c_p]),
    "ctmi_sart_residual": (c_int, [c_p, c_p, c_p, c_p, c_i64, c_p]),
    "ctmi_sart_update": (c_int, [c_p, c_p, c_p, c_i64, c_f, c_int, c_p]),
    "ctmi_em_ratio": (c_int, [c_p, c_p, c_p, c_i64, c_p]),
    "ctmi_awtv_grad": (c_int, [c_p, c_p, c_i64, c_i64, c_i64, c_f, c_f, c_p]),
    "ctmi_tv_step": (c_int, [c_p, c_p, c_i64, c_p, c_f, c_p]),
    "ctmi_em_update": (c_int, [c_p, c_p, c_p, c_i64, c_p]),
    "ctmi_fov_sq_err": (c_int, [c_p, c_p, c_p, c_p, c_p, ctypes.c_size_t, c_p]),
    "ctmi_flatten_curved": (c_int, [c_p, c_p, c_p, c_p, c_i64, c_i64, c_p]),
    "ctmi_ceiling_copy": (c_int, [c_p, c_p, c_i64, c_p]),
    "ctmi_ceiling_fma_per_lane": (c_i64, [c_int]),
    "ctmi_ceiling_fma": (c_int, [c_p, c_int, c_int, c_p]),
    # learned prior (ctmi_unet.h)
    "ctmi_conv3d_bf16_fwd": (c_int, [c_int] * 4 + [c_p, c_int, c_int, c_p, c_int, c_int, c_p, c_p, c_int, c_int, c_p,
                                                   c_int, c_p]),
    "ctmi_conv3d_bf16_dgrad": (c_int, [c_int] * 4 + [c_p, c_int, c_int, c_p, c_int, c_p, c_int, c_p, c_int, c_p]),
    "ctmi_conv3d_wgrad_workspace_bytes": (ctypes.c_size_t, [c_int] * 6),
    "ctmi_conv3d_bf16_wgrad": (c_int, [c_int] * 4 + [c_p, c_int, c_int, c_p, c_int, c_int, c_p, c_int, c_int, c_p, c_p,
                                                     c_int, c_p, ctypes.c_size_t, c_p]),
    "ctmi_conv3d_pack_weights": (c_int, [c_p, c_int, c_int, c_p, c_p, c_p]),
    "ctmi_unet_pack_input": (c_int, [c_p, c_i64, c_p, c_p]),
    "ctmi_pool2": (c_int, [c_int] * 5 + [c_p, c_int, c_p, c_int, c_p]),
    "ctmi_pool2_skip_grad": (c_int, [c_int] * 5 + [c_p, c_int, c_p, c_int, c_p, c_int, c_p, c_int, c_p]),
    "ctmi_upsample2": (c_int, [c_int] * 4 + [c_p, c_int, c_int, c_p, c_p, c_int, c_p, c_int, c_p]),
    "ctmi_upsample2_dgrad": (c_int, [c_int] * 4 + [c_p, c_int, c_int, c_p, c_int, c_p, c_int, c_p, c_int, c_p]),
    "ctmi_upsample2_wgrad_workspace_bytes": (ctypes.c_size_t, [c_int] * 6),
    "ctmi_upsample2_wgrad": (c_int, [c_int] * 4 + [c_p, c_int, c_int, c_p, c_int, c_int, c_p, c_p, c_int, c_p,
                                                   ctypes.c_size_t, c_p]),
    "ctmi_unet_head": (c_int, [c_i64, c_p, c_p, c_int, c_int, c_p, c_p, c_p, c_p]),
    "ctmi_unet_head_workspace_bytes": (ctypes.c_size_t, []),
    "ctmi_unet_head_mse_bwd": (c_int, [c_i64, c_p, c_p, c_p, c_int, c_p, c_p, c_int, c_p, c_p, c_p, ctypes.c_size_t,
                                       c_p]),
    "ctmi_adam_step": (c_int, [c_p, c_p, c_p, c_p, c_i64, c_f, c_f, c_f, c_f, c_i64, c_p]),
    "ctmi_to_bf16": (c_int, [c_p, c_i64, c_p, c_p]),
}

EXPORTED = tuple(_SIGS)

_lib = None


class CtmiError(RuntimeError):
    pass


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2412_10129_amd/build.py "
                              "(or __graft_entry__.build()) first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc == CTMI_OK:
        return
    msg = lib().ctmi_last_error().decode()
    if rc == CTMI_EINVAL:
        raise ValueError(msg)
    if rc == CTMI_EUNSUPPORTED:
        raise NotImplementedError(msg)
    raise CtmiError(f"ctmi error {rc}: {msg}")
