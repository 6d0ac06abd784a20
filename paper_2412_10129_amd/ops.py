"""Tensor-level wrappers of the libctmi entry points.

PyTorch provides device memory and the current stream; every computation is a
libctmi kernel.  Tensors must be float32, contiguous and on the plan's device.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib as L

_PROJ = {"siddon": L.CTMI_SIDDON, "interp": L.CTMI_INTERP}
_BP = {"siddon": L.CTMI_BP_SIDDON, "interp": L.CTMI_BP_INTERP, "fdk": L.CTMI_BP_FDK}
_BP_OP = {"siddon": L.CTMI_OP_BACKPROJECT_SIDDON, "interp": L.CTMI_OP_BACKPROJECT_INTERP,
          "fdk": L.CTMI_OP_BACKPROJECT_FDK}


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor, name: str, numel: Optional[int] = None, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32 (got {t.dtype})")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the plan on {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def geometry_check(geo, angles) -> None:
    a = np.ascontiguousarray(angles, dtype=np.float64)
    g = L.geometry_struct(geo)
    L.check(L.lib().ctmi_geometry_check(ctypes.byref(g), a.ctypes.data_as(ctypes.c_void_p), len(a)))


def view_table(geo, angles) -> np.ndarray:
    a = np.ascontiguousarray(angles, dtype=np.float64)
    g = L.geometry_struct(geo)
    out = np.zeros((len(a), 32), dtype=np.float32)
    L.check(L.lib().ctmi_view_table(ctypes.byref(g), a.ctypes.data_as(ctypes.c_void_p), len(a),
                                    out.ctypes.data_as(ctypes.c_void_p)))
    return out


class Plan:
    """A cone-beam geometry and its angles, resident on one GPU."""

    def __init__(self, geo, angles, device=None):
        """angles: z1 angles of a circular orbit (rad), or a per-view
        geometry description (an object with per-view arrays angles (n, 3),
        DSO, DSD, offOrigin, offDetector, COR, rotDetector; the FDK pieces
        then refuse the plan)."""
        self.geo = geo
        self.views = angles if hasattr(angles, "rotDetector") else None
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.vol_shape = tuple(int(v) for v in geo.nVoxel)
        self.det_shape = tuple(int(v) for v in geo.nDetector)
        g = L.geometry_struct(geo)
        h = ctypes.c_void_p()
        if self.views is None:
            self.angles = np.ascontiguousarray(angles, dtype=np.float64)
            self.nviews = len(self.angles)
            with torch.cuda.device(self.device):
                L.check(L.lib().ctmi_plan_create(ctypes.byref(g), self.angles.ctypes.data_as(ctypes.c_void_p),
                                                 self.nviews, ctypes.byref(h)))
        else:
            tab = L.view_structs(self.views)
            self.nviews = len(tab)
            self.angles = np.ascontiguousarray(np.asarray(self.views.angles, dtype=np.float64).reshape(-1, 3)[:, 0])
            with torch.cuda.device(self.device):
                L.check(L.lib().ctmi_plan_create_views(ctypes.byref(g), tab, self.nviews, ctypes.byref(h)))
        self._h = h
        self._ws = torch.empty(L.lib().ctmi_reduce_workspace_bytes(0) // 8, dtype=torch.float64, device=self.device)
        self._ws_bytes = {}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            with torch.cuda.device(self.device):
                L.check(L.lib().ctmi_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --------------------------------------------------------------- sizes
    def proj_shape(self, nviews: Optional[int] = None):
        return (self.nviews if nviews is None else nviews,) + self.det_shape

    def _range(self, view0, nviews):
        if nviews is None:
            nviews = self.nviews - view0
        return int(view0), int(nviews)

    # ----------------------------------------------------------- operators
    def forward(self, vol: torch.Tensor, out: Optional[torch.Tensor] = None, kind: str = "siddon", view0: int = 0,
                nviews: Optional[int] = None, stream=None) -> torch.Tensor:
        """out = A vol for views [view0, view0 + nviews)."""
        view0, nviews = self._range(view0, nviews)
        if out is None:
            out = torch.empty(self.proj_shape(nviews), dtype=torch.float32, device=self.device)
        pv = _ptr(vol, "vol", int(np.prod(self.vol_shape)), self.device)
        po = _ptr(out, "proj", nviews * self.det_shape[0] * self.det_shape[1], self.device)
        L.check(L.lib().ctmi_forward(self._h, _PROJ[kind], pv, po, view0, nviews, _stream(stream)))
        return out

    def workspace_size(self, op: int) -> int:
        """Device workspace bytes of a libctmi operation (CTMI_OP_*) on this plan."""
        n = ctypes.c_size_t()
        L.check(L.lib().ctmi_workspace_size(self._h, int(op), ctypes.byref(n)))
        return int(n.value)

    def backproject(self, proj: torch.Tensor, out: Optional[torch.Tensor] = None, kind: str = "siddon",
                    beta: float = 0.0, view0: int = 0, nviews: Optional[int] = None, stream=None,
                    ws: Optional[torch.Tensor] = None) -> torch.Tensor:
        """out = beta * out + B proj; kind 'siddon'/'interp' = matched A^T, 'fdk' = FDK backprojector.
        The workspace (interpolated A^T only) comes from torch's caching
        allocator on the call's stream unless `ws` (a device tensor of at
        least workspace_size bytes) is given."""
        view0, nviews = self._range(view0, nviews)
        if out is None:
            out = torch.empty(self.vol_shape, dtype=torch.float32, device=self.device)
            beta = 0.0
        pp = _ptr(proj, "proj", nviews * self.det_shape[0] * self.det_shape[1], self.device)
        po = _ptr(out, "vol", int(np.prod(self.vol_shape)), self.device)
        nbytes = self._ws_bytes.get(kind)
        if nbytes is None:
            nbytes = self._ws_bytes[kind] = self.workspace_size(_BP_OP[kind])
        if nbytes and ws is None:
            with torch.cuda.stream(stream) if stream is not None else _nullctx():
                ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        wp = ctypes.c_void_p(ws.data_ptr()) if ws is not None else ctypes.c_void_p()
        wb = ws.numel() * ws.element_size() if ws is not None else 0
        L.check(L.lib().ctmi_backproject(self._h, _BP[kind], pp, po, view0, nviews, float(beta), wp, wb,
                                         _stream(stream)))
        return out

    def fdk_filter(self, proj: torch.Tensor, out: Optional[torch.Tensor] = None, wang: bool = False, view0: int = 0,
                   nviews: Optional[int] = None, stream=None) -> torch.Tensor:
        view0, nviews = self._range(view0, nviews)
        if out is None:
            out = torch.empty(self.proj_shape(nviews), dtype=torch.float32, device=self.device)
        n = nviews * self.det_shape[0] * self.det_shape[1]
        L.check(L.lib().ctmi_fdk_filter(self._h, 1 if wang else 0, _ptr(proj, "proj", n, self.device),
                                        _ptr(out, "out", n, self.device), view0, nviews, _stream(stream)))
        return out

    def flatten_curved(self, curved: torch.Tensor, cd, out: Optional[torch.Tensor] = None, view0: int = 0,
                       nviews: Optional[int] = None, stream=None) -> torch.Tensor:
        """Flattening transformation: projections on the curved detector `cd`
        (nDetector, dDetector, radius, offDetector) resampled onto this
        plan's flat detector."""
        view0, nviews = self._range(view0, nviews)
        if out is None:
            out = torch.empty(self.proj_shape(nviews), dtype=torch.float32, device=self.device)
        c = L.curved_struct(cd)
        nc = nviews * int(cd.nDetector[0]) * int(cd.nDetector[1])
        L.check(L.lib().ctmi_flatten_curved(self._h, ctypes.byref(c), _ptr(curved, "curved", nc, self.device),
                                            _ptr(out, "flat", nviews * self.det_shape[0] * self.det_shape[1],
                                                 self.device), view0, nviews, _stream(stream)))
        return out

    # ---------------------------------------------------------- reductions
    def fov_sq_err(self, x: torch.Tensor, gt: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
        """out[0:2] (float64 device) = (sum of squared error, count) inside the FOV cylinder."""
        n = int(np.prod(self.vol_shape))
        L.check(L.lib().ctmi_fov_sq_err(self._h, _ptr(x, "x", n, self.device), _ptr(gt, "gt", n, self.device),
                                        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(self._ws.data_ptr()),
                                        self._ws.numel() * 8, _stream(stream)))
        return out


class _nullctx:
    def __enter__(self):
        return self

    def __exit__(self, *exc):
        return False


def stream_check(stream=None) -> None:
    """Raise if the device reported an asynchronous error on `stream` (or an
    earlier launch failed)."""
    L.check(L.lib().ctmi_stream_check(_stream(stream)))


def _ws(device):
    return torch.empty(L.lib().ctmi_reduce_workspace_bytes(0) // 8, dtype=torch.float64, device=device)


def dot(a: torch.Tensor, b: torch.Tensor, out: Optional[torch.Tensor] = None, ws=None, stream=None) -> torch.Tensor:
    """FP64 dot product on the device; returns a 1-element float64 device tensor."""
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=a.device)
    ws = _ws(a.device) if ws is None else ws
    L.check(L.lib().ctmi_dot(_ptr(a, "a"), _ptr(b, "b", a.numel()), a.numel(), ctypes.c_void_p(out.data_ptr()),
                             ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(), _stream(stream)))
    return out


def axpby(a: float, x: torch.Tensor, b: float, y: torch.Tensor, stream=None) -> torch.Tensor:
    L.check(L.lib().ctmi_axpby(y.numel(), float(a), _ptr(x, "x", y.numel()), float(b), _ptr(y, "y"), _stream(stream)))
    return y


def cgls_xr(x, p, r, q, gamma, delta, rnorm2, ws, stream=None):
    L.check(L.lib().ctmi_cgls_xr(_ptr(x, "x"), _ptr(p, "p", x.numel()), x.numel(), _ptr(r, "r"),
                                 _ptr(q, "q", r.numel()), r.numel(), ctypes.c_void_p(gamma), ctypes.c_void_p(delta),
                                 ctypes.c_void_p(rnorm2), ctypes.c_void_p(ws.data_ptr()),
                                 ws.numel() * ws.element_size(), _stream(stream)))


def cgls_p(p, s, gamma_old, gamma_new, stream=None):
    L.check(L.lib().ctmi_cgls_p(_ptr(p, "p"), _ptr(s, "s", p.numel()), p.numel(), ctypes.c_void_p(gamma_old),
                                ctypes.c_void_p(gamma_new), _stream(stream)))


def recip_or_zero(x: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    out = x if out is None else out
    L.check(L.lib().ctmi_recip_or_zero(_ptr(x, "in"), _ptr(out, "out", x.numel()), x.numel(), _stream(stream)))
    return out


def sart_residual(b, ax, w, out, stream=None):
    n = b.numel()
    L.check(L.lib().ctmi_sart_residual(_ptr(b, "b"), _ptr(ax, "ax", n), _ptr(w, "w", n), _ptr(out, "out", n), n,
                                       _stream(stream)))
    return out


def sart_update(x, v, bp, lam=1.0, nonneg=True, stream=None):
    n = x.numel()
    L.check(L.lib().ctmi_sart_update(_ptr(x, "x"), _ptr(v, "v", n), _ptr(bp, "bp", n), n, float(lam),
                                     1 if nonneg else 0, _stream(stream)))
    return x


def em_ratio(b, ax, out, stream=None):
    """out = b / ax where ax > 0, else 0 (MLEM/OSEM ratio)."""
    n = b.numel()
    L.check(L.lib().ctmi_em_ratio(_ptr(b, "b"), _ptr(ax, "ax", n), _ptr(out, "out", n), n, _stream(stream)))
    return out


def em_update(x, v, bp, stream=None):
    """x = x * v * bp (MLEM/OSEM update, v = 1 / (A^T 1))."""
    n = x.numel()
    L.check(L.lib().ctmi_em_update(_ptr(x, "x"), _ptr(v, "v", n), _ptr(bp, "bp", n), n, _stream(stream)))
    return x


def awtv_grad(x: torch.Tensor, out: Optional[torch.Tensor] = None, delta: float = float("inf"), eps: float = 1e-8,
              stream=None) -> torch.Tensor:
    """Gradient of the (adaptive-weighted) total variation of a [nz, ny, nx]
    volume, weights lagged; plain TV for delta = inf."""
    if x.dim() != 3:
        raise ValueError("x must be a [nz, ny, nx] volume")
    out = torch.empty_like(x) if out is None else out
    nz, ny, nx = x.shape
    L.check(L.lib().ctmi_awtv_grad(_ptr(x, "x"), _ptr(out, "g", x.numel()), nz, ny, nx, float(delta), float(eps),
                                   _stream(stream)))
    return out


def tv_step(x: torch.Tensor, g: torch.Tensor, gnorm2: torch.Tensor, step: float, stream=None) -> torch.Tensor:
    """x -= step * g / sqrt(gnorm2) (gnorm2: 1-element float64 device tensor)."""
    L.check(L.lib().ctmi_tv_step(_ptr(x, "x"), _ptr(g, "g", x.numel()), x.numel(),
                                 ctypes.c_void_p(gnorm2.data_ptr()), float(step), _stream(stream)))
    return x
