"""FP64 CPU oracle for the cone-beam projector hot path -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and
this package never imports the product: the two share nothing but the
seeded input generators in ``synth``.

The heavy ray operators are plain C (``ctoracle.c``, FP64, OpenMP); the
iterative methods are written here in numpy, step by step, in the paper's
order.  Every function names the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

from synth import Ellipsoid, Geometry, Views

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ctoracle.c")
_LIB = os.path.join(_HERE, "libctoracle.so")

SIDDON, INTERP = 0, 1
_KINDS = {"siddon": SIDDON, "interp": INTERP}


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Geo(ctypes.Structure):
    _fields_ = [("DSD", ctypes.c_double), ("DSO", ctypes.c_double),
                ("nz", ctypes.c_int64), ("ny", ctypes.c_int64), ("nx", ctypes.c_int64),
                ("dz", ctypes.c_double), ("dy", ctypes.c_double), ("dx", ctypes.c_double),
                ("oz", ctypes.c_double), ("oy", ctypes.c_double), ("ox", ctypes.c_double),
                ("nv", ctypes.c_int64), ("nu", ctypes.c_int64),
                ("dv", ctypes.c_double), ("du", ctypes.c_double),
                ("ov", ctypes.c_double), ("ou", ctypes.c_double),
                ("accuracy", ctypes.c_double)]


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB)
        _lib.orc_wang_weight.restype = ctypes.c_double
    return _lib


def _geo(g: Geometry) -> _Geo:
    return _Geo(g.DSD, g.DSO, *g.nVoxel, *g.dVoxel, *g.offOrigin, *g.nDetector, *g.dDetector,
                *g.offDetector, g.accuracy)


class _View(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("z1", "y1", "z2", "DSO", "DSD", "oz", "oy", "ox", "ov", "ou", "cor",
                                               "roll", "pitch", "yaw")]


class _Mode:
    """Circular views (angles: 1-D z1 array) or per-view frames (synth.Views):
    the C oracle takes the frames through orc_set_views for the duration of
    one call; the volume box is then centred at the origin and each view's
    rays are expressed relative to its own volume centre."""

    def __init__(self, geo: Geometry, angles):
        self.views = angles if isinstance(angles, Views) else None
        if self.views is None:
            self.angles = _f64(angles)
            self.g = _geo(geo)
        else:
            v = self.views
            n = len(v)
            self.angles = np.zeros(n)
            self.g = _geo(dataclasses.replace(geo, offOrigin=(0.0, 0.0, 0.0)))
            self.tab = (_View * n)()
            for k in range(n):
                self.tab[k] = _View(*v.angles[k], v.DSO[k], v.DSD[k], *v.offOrigin[k], *v.offDetector[k], v.COR[k],
                                    *v.rotDetector[k])

    def __len__(self):
        return len(self.angles)

    def __enter__(self):
        if self.views is not None:
            _L().orc_set_views(self.tab, ctypes.c_int64(len(self.angles)))
        return self

    def __exit__(self, *exc):
        if self.views is not None:
            _L().orc_set_views(None, ctypes.c_int64(0))
        return False


def _angles(angles):
    """Keep per-view Views as they are; z1 angles as float64."""
    return angles if isinstance(angles, Views) else _f64(angles)


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int64)


def num_threads() -> int:
    return int(_L().orc_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP thread count of the following oracle calls."""
    _L().orc_set_num_threads(ctypes.c_int(int(n)))


# ------------------------------------------------------------- operators
def forward(geo: Geometry, angles, vol, kind: str = "siddon") -> np.ndarray:
    """b = A x (the paper's linear model, section 2.1, Eq. 1)."""
    vol = _f64(vol).reshape(geo.nVoxel)
    with _Mode(geo, angles) as m:
        out = np.zeros((len(m),) + tuple(geo.nDetector), dtype=np.float64)
        _L().orc_forward(ctypes.byref(m.g), _KINDS[kind], _p(m.angles), ctypes.c_int64(len(m)), _p(vol), _p(out))
    return out


def backward(geo: Geometry, angles, proj, kind: str = "siddon") -> np.ndarray:
    """x = A^T y, the exact transpose of `forward` (ray-driven scatter)."""
    with _Mode(geo, angles) as m:
        proj = _f64(proj).reshape((len(m),) + tuple(geo.nDetector))
        out = np.zeros(geo.nVoxel, dtype=np.float64)
        _L().orc_backward(ctypes.byref(m.g), _KINDS[kind], _p(m.angles), ctypes.c_int64(len(m)), _p(proj), _p(out))
    return out


def forward_rays(geo: Geometry, angles, vol, views, ivs, ius, kind: str = "siddon") -> np.ndarray:
    """(A x)_i for the listed rays only (sampled parity at full size)."""
    vol = _f64(vol).reshape(geo.nVoxel)
    views, ivs, ius = _i64(views), _i64(ivs), _i64(ius)
    out = np.zeros(len(views), dtype=np.float64)
    with _Mode(geo, angles) as m:
        _L().orc_forward_rays(ctypes.byref(m.g), _KINDS[kind], _p(m.angles), _p(vol), ctypes.c_int64(len(views)),
                              _p(views), _p(ivs), _p(ius), _p(out))
    return out


def adjoint_voxels(geo: Geometry, angles, proj, iz, iy, ix, kind: str = "siddon") -> np.ndarray:
    """(A^T y)_j for the listed voxels, each matrix entry evaluated from its
    definition (cell chord, or tent sum) by brute force over the voxel's
    detector footprint."""
    iz, iy, ix = _i64(iz), _i64(iy), _i64(ix)
    out = np.zeros(len(iz), dtype=np.float64)
    fn = _L().orc_siddon_adjoint_voxels if kind == "siddon" else _L().orc_interp_adjoint_voxels
    with _Mode(geo, angles) as m:
        proj = _f64(proj).reshape((len(m),) + tuple(geo.nDetector))
        fn(ctypes.byref(m.g), _p(m.angles), ctypes.c_int64(len(m)), _p(proj), ctypes.c_int64(len(iz)),
           _p(iz), _p(iy), _p(ix), _p(out))
    return out


def gradient_voxels(geo: Geometry, angles, x, y, iz, iy, ix, kind: str = "siddon") -> np.ndarray:
    """2 (A^T (A x - y))_j for the listed voxels, each term from its
    definition: the voxel's footprint rays, their full ray sums and the
    matrix entries a_ij."""
    x = _f64(x).reshape(geo.nVoxel)
    iz, iy, ix = _i64(iz), _i64(iy), _i64(ix)
    out = np.zeros(len(iz), dtype=np.float64)
    with _Mode(geo, angles) as m:
        y = _f64(y).reshape((len(m),) + tuple(geo.nDetector))
        _L().orc_gradient_voxels(ctypes.byref(m.g), _KINDS[kind], _p(m.angles), ctypes.c_int64(len(m)), _p(x),
                                 _p(y), ctypes.c_int64(len(iz)), _p(iz), _p(iy), _p(ix), _p(out))
    return out


def dense_matrix(geo: Geometry, angles, kind: str = "siddon") -> np.ndarray:
    """Explicit system matrix, every entry from its definition (tiny sizes)."""
    with _Mode(geo, angles) as m:
        M = np.zeros((geo.n_proj(len(m)), geo.n_vox), dtype=np.float64)
        _L().orc_dense_matrix(ctypes.byref(m.g), _KINDS[kind], _p(m.angles), ctypes.c_int64(len(m)), _p(M))
    return M


def ray_endpoints(geo: Geometry, theta: float, iv: float, iu: float):
    """Source and pixel-centre positions (world mm) of ray (theta, iv, iu)."""
    S = np.zeros(3)
    P = np.zeros(3)
    g = _geo(geo)
    _L().orc_ray_endpoints(ctypes.byref(g), ctypes.c_double(theta), ctypes.c_double(iv), ctypes.c_double(iu),
                           _p(S), _p(P))
    return S, P


# ------------------------------------------------------------------- FDK
def bfdk(geo: Geometry, angles, proj) -> np.ndarray:
    """FDK backprojector: sum over views of (DSO/U)^2 times the bilinear
    detector sample where the source-voxel ray meets the detector (FDK, the
    paper's list of direct methods in section 2.1)."""
    if isinstance(angles, Views):
        raise ValueError("the FDK backprojector is defined for the circular orbit")
    angles = _f64(angles)
    proj = _f64(proj).reshape((len(angles),) + tuple(geo.nDetector))
    out = np.zeros(geo.nVoxel, dtype=np.float64)
    g = _geo(geo)
    _L().orc_bfdk(ctypes.byref(g), _p(angles), ctypes.c_int64(len(angles)), _p(proj), _p(out))
    return out


def bfdk_voxels(geo: Geometry, angles, proj, iz, iy, ix) -> np.ndarray:
    """The FDK backprojector at the listed voxels only."""
    if isinstance(angles, Views):
        raise ValueError("the FDK backprojector is defined for the circular orbit")
    angles = _f64(angles)
    proj = _f64(proj).reshape((len(angles),) + tuple(geo.nDetector))
    iz, iy, ix = _i64(iz), _i64(iy), _i64(ix)
    out = np.zeros(len(iz), dtype=np.float64)
    g = _geo(geo)
    _L().orc_bfdk_voxels(ctypes.byref(g), _p(angles), ctypes.c_int64(len(angles)), _p(proj), ctypes.c_int64(len(iz)),
                         _p(iz), _p(iy), _p(ix), _p(out))
    return out


def fdk_filter(geo: Geometry, proj, ntotal: Optional[int] = None, wang: bool = False) -> np.ndarray:
    """Cosine weight, optional Wang weight, Ram-Lak ramp (direct linear
    convolution), angular scale."""
    proj = _f64(proj)
    nviews = proj.shape[0]
    out = np.zeros_like(proj)
    g = _geo(geo)
    _L().orc_fdk_filter(ctypes.byref(g), ctypes.c_int64(nviews), ctypes.c_int64(ntotal or nviews),
                        ctypes.c_int(1 if wang else 0), _p(proj), _p(out))
    return out


def wang_weight(geo: Geometry, u: float) -> float:
    g = _geo(geo)
    return float(_L().orc_wang_weight(ctypes.byref(g), ctypes.c_double(u)))


def fdk(geo: Geometry, angles, proj, wang: bool = False) -> np.ndarray:
    """FDK reconstruction = B_FDK(filter(proj))."""
    q = fdk_filter(geo, proj, len(angles), wang)
    return bfdk(geo, angles, q)


# ----------------------------------------------------- iterative methods
def cgls(geo: Geometry, angles, b, niter: int, kind: str = "interp", x_gt=None, mask=None, callback=None):
    """CGLS (Hestenes & Stiefel; the paper's Krylov methods, section 2.2.1).

    x0 = 0; r = b - A x0; s = A^T r; p = s; gamma = |s|^2.  Each iteration:
    q = A p; delta = |q|^2 (stop if 0); alpha = gamma / delta; x += alpha p;
    r -= alpha q; s = A^T r; gamma' = |s|^2; beta = gamma'/gamma;
    p = s + beta p.  Records |r_k| (the residual-norm history) and, given a
    ground truth, |x_gt - x_k| and the PSNR (the error-norm history).
    callback(k, x), when given, sees the iterate after iteration k (1-based).
    """
    b = _f64(b)
    x = np.zeros(geo.nVoxel)
    r = b.copy()
    s = backward(geo, angles, r, kind)
    p = s.copy()
    gamma = float(np.dot(s.ravel(), s.ravel()))
    hist = {"resid": [], "err": [], "psnr": [], "alpha": [], "beta": [], "stopped": None}
    for k in range(niter):
        q = forward(geo, angles, p, kind)
        delta = float(np.dot(q.ravel(), q.ravel()))
        if delta == 0.0 or gamma == 0.0:
            hist["stopped"] = k
            break
        alpha = gamma / delta
        x = x + alpha * p
        r = r - alpha * q
        s = backward(geo, angles, r, kind)
        gamma_new = float(np.dot(s.ravel(), s.ravel()))
        beta = gamma_new / gamma
        p = s + beta * p
        gamma = gamma_new
        hist["alpha"].append(alpha)
        hist["beta"].append(beta)
        hist["resid"].append(float(np.linalg.norm(r.ravel())))
        if x_gt is not None:
            hist["err"].append(float(np.linalg.norm((x - x_gt).ravel())))
            hist["psnr"].append(psnr(x, x_gt, mask))
        if callback is not None:
            callback(k + 1, x)
    return x, hist


def pnp_cgls(geo: Geometry, angles, b, niter: int, denoiser, every: int = 5, ratio: float = 1.05,
             kind: str = "interp", x_gt=None, mask=None):
    """CGLS with a plug-and-play denoiser (the learned prior used inside the
    paper's Krylov solvers, section 2.2.1; the combination is ours).

    Runs CGLS from x = 0.  After every `every` iterations it proposes
    x' = denoiser(x) and computes r' = b - A x'.  The proposal is accepted
    when |r'| <= ratio |r|, r the CGLS residual vector; CGLS then restarts
    at x' (r = r', s = p = A^T r', gamma = |s|^2).  A rejected proposal
    changes nothing: CGLS continues as if it had not been made, so with a
    denoiser that is always rejected the iterates are those of `cgls`.
    Returns (x, hist) with the per-iteration residual norms |r_k|, the
    proposals' ratios |r'| / |r| and decisions, and the PSNR history when
    x_gt is given.
    """
    b = _f64(b)
    x = np.zeros(geo.nVoxel)
    r = b.copy()
    s = backward(geo, angles, r, kind)
    p = s.copy()
    gamma = float(np.dot(s.ravel(), s.ravel()))
    hist = {"resid": [], "psnr": [], "ratios": [], "accepted": []}
    for k in range(niter):
        if gamma > 0.0:
            q = forward(geo, angles, p, kind)
            delta = float(np.dot(q.ravel(), q.ravel()))
            alpha = gamma / delta if delta > 0.0 else 0.0
            x = x + alpha * p
            r = r - alpha * q
            s = backward(geo, angles, r, kind)
            gamma_new = float(np.dot(s.ravel(), s.ravel()))
            beta = gamma_new / gamma
            p = s + beta * p
            gamma = gamma_new
        if (k + 1) % every == 0:
            xd = _f64(denoiser(x))
            rd = b - forward(geo, angles, xd, kind)
            nr = float(np.linalg.norm(r.ravel()))
            q_ = float(np.linalg.norm(rd.ravel())) / nr if nr > 0.0 else math.inf
            hist["ratios"].append(q_)
            acc = q_ <= ratio
            hist["accepted"].append(bool(acc))
            if acc:
                x, r = xd, rd
                s = backward(geo, angles, r, kind)
                p = s.copy()
                gamma = float(np.dot(s.ravel(), s.ravel()))
        hist["resid"].append(float(np.linalg.norm(r.ravel())))
        if x_gt is not None:
            hist["psnr"].append(psnr(x, x_gt, mask))
    return x, hist


def subsets(nviews: int, blocksize: int):
    """Consecutive view blocks visited in order (the paper's ordered
    subsets, section 2.2.2, sequential ordering)."""
    return [np.arange(s, min(s + blocksize, nviews)) for s in range(0, nviews, blocksize)]


def _recip0(a):
    out = np.zeros_like(a)
    nz = a != 0
    out[nz] = 1.0 / a[nz]
    return out


def os_sart(geo: Geometry, angles, b, niter: int, blocksize: int, lam: float = 1.0, nonneg: bool = True,
            kind: str = "interp", x0=None, callback=None):
    """OS-SART (ordered-subset step of section 2.2.2 with the row/column
    length normalisation of SART).  The OS step is printed with the residual
    as (A_s x - b_s); read as (b_s - A_s x), the descent direction.

    Per block s: W = 1 / (A_s 1), V = 1 / (A_s^T 1) (0 where the sum is 0);
    x <- x + lam * V (A_s^T (W (b_s - A_s x))); then x <- max(x, 0) if nonneg.
    One iteration is one pass over all blocks.  SART is blocksize 1, SIRT
    one block.  callback(k, x), when given, sees the iterate after pass k
    (1-based).
    """
    angles = _angles(angles)
    b = _f64(b)
    x = np.zeros(geo.nVoxel) if x0 is None else _f64(x0).copy()
    blocks = subsets(len(angles), blocksize)
    W, V = [], []
    for idx in blocks:
        a = angles[idx]
        W.append(_recip0(forward(geo, a, np.ones(geo.nVoxel), kind)))
        V.append(_recip0(backward(geo, a, np.ones((len(idx),) + tuple(geo.nDetector)), kind)))
    for it in range(niter):
        for s, idx in enumerate(blocks):
            a = angles[idx]
            e = b[idx] - forward(geo, a, x, kind)
            x = x + lam * V[s] * backward(geo, a, W[s] * e, kind)
            if nonneg:
                x = np.maximum(x, 0.0)
        if callback is not None:
            callback(it + 1, x)
    return x


def osem(geo: Geometry, angles, b, niter: int, blocksize: Optional[int] = None, kind: str = "interp", x0=None):
    """MLEM and its ordered-subsets form OSEM (section 2.2, the MLEM update
    for the Kullback-Leibler data term; its OS counterpart, section 2.2.2).

    The printed update divides x by "A 1"; a volume can only be divided by
    the volume-sized column sums, so the normaliser is read as the
    sensitivity A^T 1 (the Shepp-Vardi update).  Per block s (MLEM: one block
    of all views):
        x <- x / (A_s^T 1) * A_s^T (b_s / (A_s x))
    with the ratio set to 0 where (A_s x)_i <= 0 and x set to 0 where
    (A_s^T 1)_j = 0.  Start x0 = 1 (EM needs a positive start).  One
    iteration is one pass over all blocks.
    """
    angles = _angles(angles)
    b = _f64(b)
    nv = len(angles)
    x = np.ones(geo.nVoxel) if x0 is None else _f64(x0).copy()
    blocks = subsets(nv, nv if blocksize is None else blocksize)
    sens = [backward(geo, angles[idx], np.ones((len(idx),) + tuple(geo.nDetector)), kind) for idx in blocks]
    for _ in range(niter):
        for s, idx in enumerate(blocks):
            a = angles[idx]
            ax = forward(geo, a, x, kind)
            ratio = np.zeros_like(ax)
            pos = ax > 0
            ratio[pos] = b[idx][pos] / ax[pos]
            bp = backward(geo, a, ratio, kind)
            x = x * _recip0(sens[s]) * bp
    return x


def poisson_loglik(geo: Geometry, angles, b, x, kind: str = "interp") -> float:
    """Poisson log-likelihood (up to a constant) of data b for image x:
    sum_i b_i log (A x)_i - (A x)_i over rays with (A x)_i > 0 (the quantity
    EM increases)."""
    ax = forward(geo, _angles(angles), _f64(x), kind)
    b = _f64(b)
    pos = ax > 0
    return float(np.sum(b[pos] * np.log(ax[pos])) - np.sum(ax))


# ----------------------------------------------------- TV and ASD-POCS
def _tv_terms(x, delta: float, wref=None):
    """Backward differences d_a(u) = x_u - x_{u - e_a} (axes z, y, x) at
    every voxel u whose three backward neighbours exist, and the adaptive
    weights w_a = exp(-(d_a / delta)^2) of the adaptive-weighted TV of
    section 2.2.3 (from wref's differences; w = 1 for delta = inf)."""
    x = _f64(x)
    c = x[1:, 1:, 1:]
    d = [c - x[:-1, 1:, 1:], c - x[1:, :-1, 1:], c - x[1:, 1:, :-1]]
    if wref is None:
        dw = d
    else:
        r = _f64(wref)
        cr = r[1:, 1:, 1:]
        dw = [cr - r[:-1, 1:, 1:], cr - r[1:, :-1, 1:], cr - r[1:, 1:, :-1]]
    if math.isinf(delta):
        w = [np.ones_like(c)] * 3
    else:
        w = [np.exp(-(a / delta) ** 2) for a in dw]
    return d, w


def awtv(x, delta: float = math.inf, eps: float = 0.0, wref=None) -> float:
    """Adaptive-weighted total variation (section 2.2.3, written there in
    2-D; here with the third axis added the same way):
        sum_u sqrt(w_z d_z^2 + w_y d_y^2 + w_x d_x^2 + eps)
    over voxels u with all three backward neighbours; plain (isotropic) TV
    for delta = inf.  eps > 0 smooths the norm at zero differences.  The
    weights are taken from wref's differences when given (x otherwise)."""
    d, w = _tv_terms(x, delta, wref)
    return float(np.sum(np.sqrt(w[0] * d[0] ** 2 + w[1] * d[1] ** 2 + w[2] * d[2] ** 2 + eps)))


def awtv_grad(x, delta: float = math.inf, eps: float = 1e-8):
    """Gradient of awtv with the weights held at their values for x (the
    adaptive weights are lagged: recomputed from the current image before
    each descent step, not differentiated).  Term u contributes
    w_a d_a / s_u to voxel u and -w_a d_a / s_u to u - e_a, with
    s_u = sqrt(sum_a w_a d_a^2 + eps); a term with s_u = 0 contributes 0."""
    x = _f64(x)
    d, w = _tv_terms(x, delta)
    s2 = w[0] * d[0] ** 2 + w[1] * d[1] ** 2 + w[2] * d[2] ** 2 + eps
    s = np.sqrt(s2)
    inv = np.zeros_like(s)
    inv[s > 0] = 1.0 / s[s > 0]
    q = [w[a] * d[a] * inv for a in range(3)]
    g = np.zeros_like(x)
    g[1:, 1:, 1:] += q[0] + q[1] + q[2]
    g[:-1, 1:, 1:] -= q[0]
    g[1:, :-1, 1:] -= q[1]
    g[1:, 1:, :-1] -= q[2]
    return g


def asd_pocs(geo: Geometry, angles, b, niter: int, blocksize: int = 1, kind: str = "interp", lam: float = 1.0,
             lam_red: float = 0.99, alpha: float = 0.002, alpha_red: float = 0.95, ng: int = 20,
             rmax: float = 0.95, eps_data: float = 0.0, delta: float = math.inf, eps_tv: float = 1e-8,
             nonneg: bool = True, x0=None, trace=None):
    """ASD-POCS and OS-ASD-POCS (the POCS class of section 2.2: a data
    step alternated with adaptive TV steepest descent, after Sidky and Pan;
    OS version with blocks of views, section 2.2.2; AwTV for finite delta,
    section 2.2.3).  Per iteration:
      1. data step: one OS-SART pass (blocks of `blocksize` views, step lam,
         x = max(x, 0) after each block if nonneg);
      2. dd = |A x - b|, dp = |x - x_before_data_step|;
         on the first iteration the TV step length is dtvg = alpha dp;
      3. ng steps x <- x - dtvg g / |g|, g = awtv_grad(x) (skipped when
         |g| = 0);
      4. dg = |x - x_before_tv|; if dg > rmax dp and dd > eps_data then
         dtvg <- dtvg alpha_red;
      5. lam <- lam lam_red.
    The paper names the algorithm and its parameters without the steps;
    these follow Sidky and Pan's published description.  When `trace` is a
    list, one dict per iteration is appended with the quantities of steps
    2-5: dp, dd, dg, the TV step length used (dtvg) and the data step used
    (lam)."""
    angles = _angles(angles)
    b = _f64(b)
    x = np.zeros(geo.nVoxel) if x0 is None else _f64(x0).copy()
    blocks = subsets(len(angles), blocksize)
    W, V = [], []
    for idx in blocks:
        a = angles[idx]
        W.append(_recip0(forward(geo, a, np.ones(geo.nVoxel), kind)))
        V.append(_recip0(backward(geo, a, np.ones((len(idx),) + tuple(geo.nDetector)), kind)))
    dtvg = None
    for k in range(niter):
        x_prev = x.copy()
        for s, idx in enumerate(blocks):
            a = angles[idx]
            e = b[idx] - forward(geo, a, x, kind)
            x = x + lam * V[s] * backward(geo, a, W[s] * e, kind)
            if nonneg:
                x = np.maximum(x, 0.0)
        dd = float(np.linalg.norm(forward(geo, angles, x, kind) - b))
        dp = float(np.linalg.norm(x - x_prev))
        if dtvg is None:
            dtvg = alpha * dp
        x_tv = x.copy()
        for _ in range(ng):
            g = awtv_grad(x, delta, eps_tv)
            gn = float(np.linalg.norm(g))
            if gn > 0:
                x = x - dtvg * g / gn
        dg = float(np.linalg.norm(x - x_tv))
        if trace is not None:
            trace.append({"dp": dp, "dd": dd, "dg": dg, "dtvg": dtvg, "lam": lam})
        if dg > rmax * dp and dd > eps_data:
            dtvg *= alpha_red
        lam *= lam_red
    return x


# ------------------------------------------------------ curved detectors
def curved_pixel_centres(geo: Geometry, theta: float, cd) -> np.ndarray:
    """World positions (nv, nu, 3) of a curved detector's pixel centres for
    the view at gantry angle theta (curved detectors, section 2.4).

    With e_s = (cos t, sin t, 0) pointing at the source S = DSO e_s,
    u_hat = (-sin t, cos t, 0) and the flat detector's centre D = S - DSD e_s,
    the arc's axis runs through A = D + R e_s parallel to z (R = cd.radius),
    and pixel (iv, iu), at arc length s = (iu + 1/2 - nu/2) du + off_u and
    height v = (iv + 1/2 - nv/2) dv + off_v, sits at
    A - R cos(s / R) e_s + R sin(s / R) u_hat + v z."""
    c, sn = math.cos(theta), math.sin(theta)
    es = np.array([c, sn, 0.0])
    uh = np.array([-sn, c, 0.0])
    zh = np.array([0.0, 0.0, 1.0])
    S = geo.DSO * es
    A = S - geo.DSD * es + cd.radius * es
    nv, nu = cd.nDetector
    s = (np.arange(nu) + 0.5 - nu / 2) * cd.dDetector[1] + cd.offDetector[1]
    v = (np.arange(nv) + 0.5 - nv / 2) * cd.dDetector[0] + cd.offDetector[0]
    phi = s / cd.radius
    row = A[None, :] - cd.radius * np.cos(phi)[:, None] * es[None, :] + cd.radius * np.sin(phi)[:, None] * uh[None, :]
    return row[None, :, :] + v[:, None, None] * zh[None, None, :]


def flatten_curved(geo: Geometry, cd, curved) -> np.ndarray:
    """The flattening transformation of the paper's curved-detector support
    (section 2.4): projections measured on the curved detector `cd` (views,
    nv_c, nu_c), resampled onto the flat detector of `geo`.

    Flat pixel (iv, iu) at (u_f, v_f) (the geometry's pixel centres) defines
    the ray from the source through D + u_f u_hat + v_f z.  In the plane
    normal to z, the point at parameter t along that ray (t = 1 on the flat
    detector) lies at (DSD - R - t DSD) e_s + t u_f u_hat from the arc's axis;
    the ray meets the cylinder where that distance is R, i.e. at the
    positive root of
        (DSD^2 + u_f^2) t^2 - 2 DSD (DSD - R) t + (DSD - R)^2 - R^2 = 0
    (one positive root: R > DSD / 2 keeps the source inside the cylinder).
    There the arc length is s = R atan2(t u_f, t DSD - DSD + R) and the
    height v = t v_f.  The flat value is the curved projection at (s, v),
    bilinear between curved pixel centres and 0 outside the curved detector:
    the ray is the same, so its line integral is carried over unchanged.
    The geometry repeats for every view of a circular orbit."""
    curved = _f64(curved)
    if not cd.radius > geo.DSD / 2:
        raise ValueError("the arc radius must exceed DSD / 2")
    nv, nu = geo.nDetector
    R, DSD = cd.radius, geo.DSD
    uf = (np.arange(nu) + 0.5 - nu / 2) * geo.dDetector[1] + geo.offDetector[1]
    vf = (np.arange(nv) + 0.5 - nv / 2) * geo.dDetector[0] + geo.offDetector[0]
    a = DSD * DSD + uf * uf
    b = -2.0 * DSD * (DSD - R)
    c = (DSD - R) ** 2 - R * R
    t = (-b + np.sqrt(b * b - 4.0 * a * c)) / (2.0 * a)
    s = R * np.arctan2(t * uf, t * DSD - DSD + R)                 # (nu,)
    vc = t[None, :] * vf[:, None]                                  # (nv, nu)
    nvc, nuc = cd.nDetector
    cu = (s - cd.offDetector[1]) / cd.dDetector[1] + nuc / 2 - 0.5
    cv = (vc - cd.offDetector[0]) / cd.dDetector[0] + nvc / 2 - 0.5
    iu0 = np.floor(cu).astype(np.int64)
    iv0 = np.floor(cv).astype(np.int64)
    fu = cu - iu0
    fv = cv - iv0
    out = np.zeros((curved.shape[0], nv, nu))
    for du_ in (0, 1):
        for dv_ in (0, 1):
            ju = np.broadcast_to(iu0 + du_, (nv, nu))
            jv = iv0 + dv_
            w = (fu if du_ else 1.0 - fu)[None, :] * (fv if dv_ else 1.0 - fv)
            ok = (ju >= 0) & (ju < nuc) & (jv >= 0) & (jv < nvc)
            out += np.where(ok, w, 0.0)[None] * curved[:, np.clip(jv, 0, nvc - 1), np.clip(ju, 0, nuc - 1)]
    return out


# --------------------------------------------------------------- metrics
def fov_mask(geo: Geometry) -> np.ndarray:
    """Voxels whose centre lies inside the volume's inscribed cylinder."""
    nz, ny, nx = geo.nVoxel
    dz, dy, dx = geo.dVoxel
    y = (np.arange(ny) + 0.5 - ny / 2) * dy
    x = (np.arange(nx) + 0.5 - nx / 2) * dx
    m2 = (y[:, None] ** 2 + x[None, :] ** 2) <= geo.iso_fov_radius() ** 2
    return np.broadcast_to(m2, (nz, ny, nx))


def psnr(x, x_gt, mask=None) -> float:
    """10 log10(R^2 / MSE) over the mask, R = the range of x_gt on the mask
    (FP64).  Judges the error-norm history of the paper's section 2.2.3."""
    x = _f64(x)
    x_gt = _f64(x_gt)
    if mask is None:
        mask = np.ones(x.shape, dtype=bool)
    d = (x - x_gt)[mask]
    mse = float(np.mean(d * d))
    g = x_gt[mask]
    R = float(g.max() - g.min())
    if mse == 0.0:
        return math.inf
    return 10.0 * math.log10(R * R / mse)


# ---------------------------------------------------- analytic phantoms
def ellipsoid_line_integrals(ellipsoids: Sequence[Ellipsoid], S: np.ndarray, P: np.ndarray) -> np.ndarray:
    """Closed-form line integrals of additive ellipsoids along segments
    S -> P (arrays (..., 3), world mm).  In the ellipsoid's normalised frame
    u = R^T (S - c) / a, w = R^T dhat / a; with A = w.w, B = u.w,
    C = u.u - 1 the chord is 2 sqrt(B^2 - AC) / A when positive."""
    S = np.asarray(S, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    d = P - S
    L = np.linalg.norm(d, axis=-1, keepdims=True)
    dh = d / L
    out = np.zeros(S.shape[:-1])
    for e in ellipsoids:
        c = np.asarray(e.c)
        a = np.asarray(e.a)
        R = np.asarray(e.R)
        u = ((S - c) @ R) / a
        w = (dh @ R) / a
        A = np.sum(w * w, -1)
        B = np.sum(u * w, -1)
        C = np.sum(u * u, -1) - 1.0
        disc = B * B - A * C
        chord = np.where(disc > 0, 2.0 * np.sqrt(np.maximum(disc, 0.0)) / A, 0.0)
        out += e.rho * chord
    return out


def analytic_projections(geo: Geometry, angles, ellipsoids: Sequence[Ellipsoid]) -> np.ndarray:
    """Closed-form cone-beam projections of an ellipsoid phantom, all rays."""
    angles = _f64(angles)
    nv, nu = geo.nDetector
    out = np.zeros((len(angles), nv, nu))
    iv, iu = np.meshgrid(np.arange(nv), np.arange(nu), indexing="ij")
    for k, th in enumerate(angles):
        c, s = math.cos(th), math.sin(th)
        u = (iu + 0.5 - nu / 2) * geo.dDetector[1] + geo.offDetector[1]
        v = (iv + 0.5 - nv / 2) * geo.dDetector[0] + geo.offDetector[0]
        S = np.array([geo.DSO * c, geo.DSO * s, 0.0])
        P = np.stack([S[0] - geo.DSD * c - u * s, S[1] - geo.DSD * s + u * c, v], -1)
        out[k] = ellipsoid_line_integrals(ellipsoids, np.broadcast_to(S, P.shape), P)
    return out
