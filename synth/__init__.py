"""Seeded synthetic inputs shared by the HIP path, the FP64 oracle and the tests.

This module only *describes* workloads and draws random inputs.  It holds
none of the projector, filter or solver arithmetic: geometry is a plain
record of the acquisition parameters (the paper's geometry table in its
appendix on geometric parameters, and the default circular cone-beam set-up
of its section on geometric flexibility), phantoms are lists of ellipsoids
plus their voxelisation, and noise is the Beer-Lambert/Poisson model that a
data loader applies to raw counts.

Conventions (fixed here, used by both sides):
  * world frame in mm; the object is static, the source rotates about +z;
  * volumes are C-order ``[nz][ny][nx]`` (x fastest); every per-axis tuple
    of the volume is ordered (z, y, x);
  * projections are C-order ``[nviews][nv][nu]`` (u fastest); every per-axis
    tuple of the detector is ordered (v, u);
  * angles are the z1 gantry angles, theta_k = 2*pi*k/N (endpoint excluded).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

__all__ = [
    "Geometry", "Ellipsoid", "WORKLOADS", "workload", "circular_angles",
    "head_phantom", "random_ellipsoids", "voxelize", "gaussian_texture",
    "uniform_volume", "uniform_projections", "poisson_log_data", "normal_weights",
    "bf16_values", "textured_phantom", "CurvedDetector",
]


@dataclasses.dataclass(frozen=True)
class Geometry:
    """Circular cone-beam geometry (the paper's geometry-parameter table).

    sVoxel and sDetector are derived (n * d); the table lists the total size
    and the element size under the same name twice, read here as total size
    (s*) and element size (d*).
    """
    DSD: float                               # source -> detector distance, mm
    DSO: float                               # source -> origin distance, mm
    nVoxel: Tuple[int, int, int]             # (nz, ny, nx)
    dVoxel: Tuple[float, float, float]       # (dz, dy, dx) mm
    nDetector: Tuple[int, int]               # (nv, nu)
    dDetector: Tuple[float, float]           # (dv, du) mm
    offOrigin: Tuple[float, float, float] = (0.0, 0.0, 0.0)   # (z, y, x) mm
    offDetector: Tuple[float, float] = (0.0, 0.0)             # (v, u) mm
    accuracy: float = 0.5                    # interpolated-projector step, voxels

    @property
    def sVoxel(self):
        return tuple(n * d for n, d in zip(self.nVoxel, self.dVoxel))

    @property
    def sDetector(self):
        return tuple(n * d for n, d in zip(self.nDetector, self.dDetector))

    @property
    def n_vox(self) -> int:
        return int(np.prod(self.nVoxel))

    def n_proj(self, nviews: int) -> int:
        return int(nviews) * int(self.nDetector[0]) * int(self.nDetector[1])

    def replace(self, **kw) -> "Geometry":
        return dataclasses.replace(self, **kw)

    def iso_fov_radius(self) -> float:
        """Radius of the volume's inscribed cylinder (the FOV mask), mm."""
        return 0.5 * min(self.nVoxel[1] * self.dVoxel[1], self.nVoxel[2] * self.dVoxel[2])


@dataclasses.dataclass(frozen=True)
class CurvedDetector:
    """A cylindrically curved detector (the paper's curved detectors, section
    2.4: the pixel rows follow an arc in the fan direction, straight along v).

    The arc passes through the flat detector's centre, with its axis parallel
    to v at distance `radius` from that centre towards the source; radius =
    DSD puts every pixel of a row at the same distance from the source.  u
    pixel positions are arc lengths from the centre.
    """
    nDetector: Tuple[int, int]          # (nv, nu)
    dDetector: Tuple[float, float]      # (dv, du) mm, du along the arc
    radius: float                       # mm
    offDetector: Tuple[float, float] = (0.0, 0.0)   # (v, u) mm, u along the arc


def circular_angles(n: int) -> np.ndarray:
    """theta_k = 2*pi*k/n, k = 0..n-1 (full orbit, no duplicated endpoint)."""
    return 2.0 * np.pi * np.arange(n, dtype=np.float64) / n


@dataclasses.dataclass(frozen=True, eq=False)
class Views:
    """Per-projection geometry (the paper's geometric flexibility: Euler ZYZ
    gantry angles, centre-of-rotation shift, in-place detector rotation, and
    every parameter except the image and detector sizes settable per
    projection).  Arrays over the views:
      angles      (n, 3) z1, y1, z2 (rad), gantry R = Rz(z1) Ry(y1) Rz(z2);
      DSO, DSD    (n,)   mm;
      offOrigin   (n, 3) z, y, x (mm) volume centre;
      offDetector (n, 2) v, u (mm), along the (rotated) detector axes;
      COR         (n,)   mm, source-detector line shifted along the machine
                         y axis (before the gantry rotation);
      rotDetector (n, 3) roll, pitch, yaw (rad) of the detector about its
                         centre: about its normal, its u axis, its v axis.
    (z1, 0, 0) with the other fields from the Geometry is the circular orbit.
    """
    angles: np.ndarray
    DSO: np.ndarray
    DSD: np.ndarray
    offOrigin: np.ndarray
    offDetector: np.ndarray
    COR: np.ndarray
    rotDetector: np.ndarray

    def __len__(self) -> int:
        return int(self.angles.shape[0])

    def __getitem__(self, idx) -> "Views":
        return Views(*(np.atleast_1d(np.asarray(getattr(self, f.name)))[idx] if f.name in ("DSO", "DSD", "COR")
                       else np.asarray(getattr(self, f.name))[idx] for f in dataclasses.fields(self)))


def views(geo: Geometry, angles, **per_view) -> Views:
    """Views from z1 angles (or (n, 3) ZYZ angles) with the Geometry's
    scalar parameters, any of which may be overridden per view."""
    a = np.asarray(angles, dtype=np.float64)
    if a.ndim == 1:
        a = np.stack([a, np.zeros_like(a), np.zeros_like(a)], axis=1)
    n = a.shape[0]

    def arr(name, default, width=None):
        v = np.asarray(per_view.get(name, default), dtype=np.float64)
        shape = (n,) if width is None else (n, width)
        return np.ascontiguousarray(np.broadcast_to(v, shape))

    unknown = set(per_view) - {"DSO", "DSD", "offOrigin", "offDetector", "COR", "rotDetector"}
    if unknown:
        raise ValueError(f"unknown per-view fields {sorted(unknown)}")
    return Views(np.ascontiguousarray(a), arr("DSO", geo.DSO), arr("DSD", geo.DSD),
                 arr("offOrigin", geo.offOrigin, 3), arr("offDetector", geo.offDetector, 2),
                 arr("COR", 0.0), arr("rotDetector", (0.0, 0.0, 0.0), 3))


# ---------------------------------------------------------------- workloads
# Five synthetic workloads.  DSO/DSD are shared; sizes follow the cone-beam
# experiment shapes (a 1024x768 detector like the clinical head scans).
_DSO, _DSD = 1000.0, 1536.0
WORKLOADS = {
    # 64^3 head phantom, Siddon + matched backprojector + FDK (Ram-Lak)
    "head64": dict(geo=Geometry(_DSD, _DSO, (64, 64, 64), (1.0, 1.0, 1.0), (64, 64), (1.6, 1.6)),
                   nviews=64),
    # 256^3 random ellipsoids, interpolated projector, CGLS-20 / OS-SART
    "ellipsoids256": dict(geo=Geometry(_DSD, _DSO, (256, 256, 256), (1.0, 1.0, 1.0), (512, 512), (0.8, 0.8)),
                          nviews=360),
    # 512^3 x 720 views, 1024x768 detector: the operator-throughput workload
    "cbct512": dict(geo=Geometry(_DSD, _DSO, (512, 512, 512), (0.5, 0.5, 0.5), (768, 1024), (0.512, 0.512)),
                    nviews=720),
    # 256^3, 90 sparse vs 720 dense views (learned-prior workload)
    "sparse256": dict(geo=Geometry(_DSD, _DSO, (256, 256, 256), (1.0, 1.0, 1.0), (512, 512), (0.8, 0.8)),
                      nviews=90, dense_nviews=720),
    # 1024^3 x 1440 views, 1536^2 detector, 20 mm lateral detector offset
    "large1024": dict(geo=Geometry(_DSD, _DSO, (1024, 1024, 1024), (0.25, 0.25, 0.25), (1536, 1536), (0.3, 0.3),
                                   offDetector=(0.0, 20.0)),
                      nviews=1440),
}


def workload(name: str):
    w = WORKLOADS[name]
    return w["geo"], circular_angles(w["nviews"])


# ----------------------------------------------------------------- phantoms
@dataclasses.dataclass(frozen=True)
class Ellipsoid:
    """Additive ellipsoid: rho * indicator(|R^T (X - c) / a| <= 1).

    c is the world centre (x, y, z) mm, a the semi-axes mm, R a 3x3 rotation
    whose columns are the ellipsoid's axes in world coordinates.
    """
    c: Tuple[float, float, float]
    a: Tuple[float, float, float]
    R: Tuple[Tuple[float, float, float], ...]
    rho: float


def _rot_z(phi: float) -> np.ndarray:
    c, s = math.cos(phi), math.sin(phi)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def _rot_y(phi: float) -> np.ndarray:
    c, s = math.cos(phi), math.sin(phi)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def head_phantom(geo: Geometry, seed: int = 1) -> List[Ellipsoid]:
    """A nested-ellipsoid head phantom in the style of the 3-D Shepp-Logan
    phantom: a dense shell, a soft interior and small low-contrast features.
    The parameters are this project's own (not the published table); every
    centre gets a seeded uniform offset in [-2, 2] mm (one offset shared by
    the shell and its interior).

    Geometry is expressed in units of the half-extent of the volume.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    hz = geo.nVoxel[0] * geo.dVoxel[0] / 2
    hy = geo.nVoxel[1] * geo.dVoxel[1] / 2
    hx = geo.nVoxel[2] * geo.dVoxel[2] / 2
    oz, oy, ox = geo.offOrigin
    #      centre (x, y, z)        semi-axes (x, y, z)      rot_z deg  rot_y deg  rho
    spec = [
        ((0.00, 0.00, 0.00), (0.70, 0.90, 0.84), 0.0, 0.0, 1.00),
        ((0.00, -0.01, 0.00), (0.66, 0.86, 0.79), 0.0, 0.0, -0.78),
        ((0.21, 0.04, 0.10), (0.09, 0.26, 0.16), -16.0, 0.0, -0.12),
        ((-0.21, 0.04, 0.10), (0.10, 0.30, 0.17), 16.0, 0.0, -0.12),
        ((0.00, 0.33, 0.05), (0.19, 0.22, 0.18), 0.0, 0.0, 0.07),
        ((0.00, 0.08, 0.05), (0.05, 0.05, 0.05), 0.0, 0.0, 0.05),
        ((0.00, -0.08, 0.05), (0.05, 0.05, 0.05), 0.0, 0.0, 0.05),
        ((-0.09, -0.58, -0.22), (0.05, 0.03, 0.04), 0.0, 0.0, 0.06),
        ((0.00, -0.60, -0.22), (0.03, 0.03, 0.03), 0.0, 0.0, 0.06),
        ((0.08, -0.58, -0.22), (0.03, 0.05, 0.04), 0.0, 0.0, 0.06),
        ((0.27, -0.32, 0.30), (0.11, 0.06, 0.12), 30.0, 20.0, 0.04),
    ]
    out = []
    shell_off = rng.uniform(-2.0, 2.0, size=3)
    for i, ((cx, cy, cz), (ax, ay, az), rz, ry, rho) in enumerate(spec):
        # the shell and its interior share one offset so that they stay nested
        off = shell_off if i < 2 else rng.uniform(-2.0, 2.0, size=3)
        c = (cx * hx + ox + off[0], cy * hy + oy + off[1], cz * hz + oz + off[2])
        a = (ax * hx, ay * hy, az * hz)
        R = _rot_z(math.radians(rz)) @ _rot_y(math.radians(ry))
        out.append(Ellipsoid(c, a, tuple(map(tuple, R)), rho))
    return out


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    # uniform random unit quaternion (Shoemake 1992)
    u1, u2, u3 = rng.uniform(size=3)
    q = np.array([math.sqrt(1 - u1) * math.sin(2 * math.pi * u2), math.sqrt(1 - u1) * math.cos(2 * math.pi * u2),
                  math.sqrt(u1) * math.sin(2 * math.pi * u3), math.sqrt(u1) * math.cos(2 * math.pi * u3)])
    x, y, z, w = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def random_ellipsoids(geo: Geometry, seed: int, count_range=(10, 30), axis_range=(5.0, 60.0),
                      rho_range=(0.0, 1.0)) -> List[Ellipsoid]:
    """10-30 random ellipsoids: semi-axes ~U(5, 60) mm, densities ~U(0, 1),
    uniform rotations; centres uniform in the region that keeps each
    ellipsoid's bounding sphere inside 0.9 x the volume's inscribed cylinder.
    Axis bounds are clipped so that this region is never empty on small
    volumes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    oz, oy, ox = geo.offOrigin
    R_cyl = 0.9 * geo.iso_fov_radius()
    H_half = 0.9 * geo.nVoxel[0] * geo.dVoxel[0] / 2
    amax_allowed = 0.8 * min(R_cyl, H_half)
    lo, hi = axis_range
    hi = min(hi, amax_allowed)
    lo = min(lo, 0.5 * hi)
    n = int(rng.integers(count_range[0], count_range[1] + 1))
    out = []
    for _ in range(n):
        a = rng.uniform(lo, hi, size=3)
        R = _random_rotation(rng)
        rho = float(rng.uniform(*rho_range))
        r = float(a.max())
        while True:
            cxy = rng.uniform(-(R_cyl - r), R_cyl - r, size=2)
            if math.hypot(cxy[0], cxy[1]) + r <= R_cyl:
                break
        cz = float(rng.uniform(-(H_half - r), H_half - r))
        out.append(Ellipsoid((cxy[0] + ox, cxy[1] + oy, cz + oz), tuple(a), tuple(map(tuple, R)), rho))
    return out


def voxelize(geo: Geometry, ellipsoids: Sequence[Ellipsoid], sub: int = 4, dtype=np.float32) -> np.ndarray:
    """Mean of sub^3 point samples of the additive indicator per voxel.

    Voxels whose centre is far inside or outside an ellipsoid (farther than
    the voxel's half-diagonal in the ellipsoid's normalised frame) take the
    exact value 0 or rho without sub-sampling."""
    nz, ny, nx = geo.nVoxel
    dz, dy, dx = geo.dVoxel
    oz, oy, ox = geo.offOrigin
    lo = np.array([ox - nx * dx / 2, oy - ny * dy / 2, oz - nz * dz / 2])
    d = np.array([dx, dy, dz])
    n = np.array([nx, ny, nz])
    vol = np.zeros((nz, ny, nx), dtype=np.float64)
    offs = (np.arange(sub) + 0.5) / sub - 0.5
    sub_off = np.stack(np.meshgrid(offs, offs, offs, indexing="ij"), -1).reshape(-1, 3) * d  # (sub^3, 3)
    half_diag = 0.5 * float(np.linalg.norm(d))
    for e in ellipsoids:
        c = np.asarray(e.c, dtype=np.float64)
        a = np.asarray(e.a, dtype=np.float64)
        R = np.asarray(e.R, dtype=np.float64)
        ext = np.abs(R) @ a + half_diag            # world bounding-box half-extent
        i0 = np.maximum(np.floor((c - ext - lo) / d).astype(int), 0)
        i1 = np.minimum(np.ceil((c + ext - lo) / d).astype(int), n)
        if np.any(i1 <= i0):
            continue
        xs = lo[0] + (np.arange(i0[0], i1[0]) + 0.5) * d[0]
        ys = lo[1] + (np.arange(i0[1], i1[1]) + 0.5) * d[1]
        zs = lo[2] + (np.arange(i0[2], i1[2]) + 0.5) * d[2]
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        P = np.stack([X, Y, Z], -1) - c                 # (..., 3)
        Q = (P @ R) / a                                 # R^T (X - c) / a
        rad = np.sqrt(np.sum(Q * Q, -1))
        margin = half_diag / a.min()
        inside = rad <= 1.0 - margin
        edge = np.abs(rad - 1.0) < margin
        frac = inside.astype(np.float64)
        if edge.any():
            Pe = P[edge]                                # (m, 3)
            S = Pe[:, None, :] + sub_off[None, :, :]    # (m, sub^3, 3)
            Qe = (S @ R) / a
            frac[edge] = np.mean(np.sum(Qe * Qe, -1) <= 1.0, axis=1)
        vol[i0[2]:i1[2], i0[1]:i1[1], i0[0]:i1[0]] += e.rho * frac
    return vol.astype(dtype)


def gaussian_texture(geo: Geometry, seed: int, support: np.ndarray, sigma_vox: float = 4.0,
                     std: float = 0.02) -> np.ndarray:
    """Smooth Gaussian texture: white N(0,1) noise filtered by a Gaussian of
    sigma voxels (FP64), scaled to the given std and masked by `support`."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal(geo.nVoxel)
    t = gaussian_filter(w, sigma_vox, mode="constant")
    t *= std / max(float(t.std()), 1e-30)
    return t * (support > 0)


def uniform_volume(geo: Geometry, seed: int, dtype=np.float32) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random(geo.nVoxel, dtype=np.float64 if dtype == np.float64 else np.float32)


def uniform_projections(geo: Geometry, nviews: int, seed: int, dtype=np.float32) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (nviews,) + tuple(geo.nDetector)
    return rng.random(shape, dtype=np.float64 if dtype == np.float64 else np.float32)


def poisson_log_data(p: np.ndarray, seed: int, I0: float = 1e5, mu_w: float = 0.02) -> np.ndarray:
    """Noisy line integrals: counts N ~ Poisson(I0 * exp(-mu_w * p)), then the
    Beer-Lambert log transform p~ = -ln(max(N, 1) / I0) / mu_w.  `mu_w`
    (mm^-1 per density unit) converts densities into attenuation."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = I0 * np.exp(-mu_w * np.asarray(p, dtype=np.float64))
    N = rng.poisson(lam)
    return (-np.log(np.maximum(N, 1) / I0) / mu_w).astype(np.asarray(p).dtype)


def normal_weights(seed: int, specs) -> List[np.ndarray]:
    """Initial network weights: for each (shape, std) in `specs`, in order,
    N(0, std^2) values from one seeded PCG64 stream, as FP32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [(rng.standard_normal(tuple(shape)) * std).astype(np.float32) for shape, std in specs]


def bf16_values(shape, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Uniform values in [lo, hi) that are exactly representable in BF16
    (FP32 numbers whose low 16 bits are zero), as FP32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.uniform(lo, hi, tuple(shape)).astype(np.float32)
    return (a.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)


def textured_phantom(geo: Geometry, seed: int, dtype=np.float32) -> np.ndarray:
    """Random-ellipsoid phantom plus a smooth texture on its support
    (Gaussian-filtered white noise, sigma 4 voxels, std 0.02), clamped at 0.
    Ellipsoids from `seed`, texture noise from seed + 1_000_000."""
    v = voxelize(geo, random_ellipsoids(geo, seed), dtype=np.float64)
    v = v + gaussian_texture(geo, seed + 1_000_000, v > 0)
    return np.maximum(v, 0.0).astype(dtype)
