"""Write the FP64 oracle's CGLS and OS-SART results on the 256^3 random-ellipsoid workload.

Test infrastructure: calls only the oracle (``oracle/``) and the seeded input
generators (``synth/``); nothing here touches the HIP library.

Workload (Krylov and ordered-subset solvers of the paper's section 2.2.1 and
2.2.2 on a cone-beam scan): 256^3 volume at 1 mm, 360 views over the full
circle, 512x512 detector at 0.8 mm, DSO 1000 mm, DSD 1536 mm, interpolated
projector with a 0.5-voxel step.  Phantom: 10-30 random ellipsoids (seed 2),
voxelised with 4^3 sub-samples and rounded to FP32 (the values both sides
start from).  Data: b = A x (FP64 oracle) with Poisson counts at I0 = 1e5
(seed 12) through the Beer-Lambert log transform.

Stored (``ellipsoids256_<alg>.npz``): the iterate at 4096 seeded voxels after
the listed iterations (CGLS) or passes (OS-SART: 20 blocks of 18 consecutive
views, nonneg), its central z and y slices after the last one, the residual
norms, step lengths and PSNR history (CGLS), the noisy and clean data at 4096
seeded rays, and the oracle's wall time and thread count.

    OMP_NUM_THREADS=6 python tests/golden/make_ellipsoids256.py [cgls|ossart|both]
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
PHANTOM_SEED, NOISE_SEED, VOXEL_SEED, RAY_SEED = 2, 12, 7, 8
I0 = 1e5
CGLS_ITERS, CGLS_KEEP = 20, (1, 2, 5, 10, 20)
SART_BLOCK, SART_PASSES, SART_KEEP = 18, 20, (1, 5, 10, 20)
NSAMPLE = 4096


def samples(geo, nviews):
    """Seeded voxel and ray samples shared with the GPU test."""
    rng = np.random.Generator(np.random.PCG64(VOXEL_SEED))
    nz, ny, nx = geo.nVoxel
    vox = np.stack([rng.integers(0, nz, NSAMPLE), rng.integers(0, ny, NSAMPLE), rng.integers(0, nx, NSAMPLE)])
    rng = np.random.Generator(np.random.PCG64(RAY_SEED))
    nv, nu = geo.nDetector
    rays = np.stack([rng.integers(0, nviews, NSAMPLE), rng.integers(0, nv, NSAMPLE), rng.integers(0, nu, NSAMPLE)])
    return vox, rays


def problem():
    geo, ang = synth.workload("ellipsoids256")
    x_gt = synth.voxelize(geo, synth.random_ellipsoids(geo, PHANTOM_SEED), dtype=np.float32).astype(np.float64)
    t = time.time()
    b_clean = oracle.forward(geo, ang, x_gt, "interp")
    t_fwd = time.time() - t
    b = synth.poisson_log_data(b_clean, NOISE_SEED, I0=I0)
    return geo, ang, x_gt, b_clean, b, t_fwd


def log(msg):
    print(time.strftime("%H:%M:%S"), msg, flush=True)


def main(which):
    geo, ang, x_gt, b_clean, b, t_fwd = problem()
    vox, rays = samples(geo, len(ang))
    iz, iy, ix = vox
    mask = oracle.fov_mask(geo)
    log(f"data ready (A {t_fwd:.0f} s, {oracle.num_threads()} threads)")
    common = dict(vox=vox, rays=rays, b_rays=b[rays[0], rays[1], rays[2]],
                  b_clean_rays=b_clean[rays[0], rays[1], rays[2]], x_gt_vox=x_gt[iz, iy, ix])
    meta = dict(phantom_seed=PHANTOM_SEED, noise_seed=NOISE_SEED, voxel_seed=VOXEL_SEED, ray_seed=RAY_SEED,
                I0=I0, threads=oracle.num_threads(), forward_s=t_fwd, workload="ellipsoids256", kind="interp")
    zc, yc = geo.nVoxel[0] // 2, geo.nVoxel[1] // 2
    if which in ("cgls", "both"):
        keep = {}

        def cb(k, x):
            log(f"cgls iteration {k}")
            if k in CGLS_KEEP:
                keep[k] = x[iz, iy, ix].copy()
        t = time.time()
        x, hist = oracle.cgls(geo, ang, b, CGLS_ITERS, "interp", x_gt=x_gt, mask=mask, callback=cb)
        dt = time.time() - t
        np.savez_compressed(os.path.join(HERE, "ellipsoids256_cgls.npz"), **common,
                            iters=np.array(CGLS_KEEP), x_vox=np.stack([keep[k] for k in CGLS_KEEP]),
                            slice_z=x[zc].astype(np.float32), slice_y=x[:, yc].astype(np.float32),
                            resid=np.array(hist["resid"]), alpha=np.array(hist["alpha"]),
                            beta=np.array(hist["beta"]), psnr=np.array(hist["psnr"]),
                            meta=json.dumps(dict(meta, iterations=CGLS_ITERS, seconds=dt)))
        log(f"cgls done in {dt:.0f} s")
    if which in ("ossart", "both"):
        keep = {}

        def cb(k, x):
            log(f"os-sart pass {k}")
            if k in SART_KEEP:
                keep[k] = x[iz, iy, ix].copy()
        t = time.time()
        x = oracle.os_sart(geo, ang, b, SART_PASSES, SART_BLOCK, lam=1.0, nonneg=True, kind="interp", callback=cb)
        dt = time.time() - t
        np.savez_compressed(os.path.join(HERE, "ellipsoids256_ossart.npz"), **common,
                            iters=np.array(SART_KEEP), x_vox=np.stack([keep[k] for k in SART_KEEP]),
                            slice_z=x[zc].astype(np.float32), slice_y=x[:, yc].astype(np.float32),
                            psnr=np.array([oracle.psnr(x, x_gt, mask)]),
                            meta=json.dumps(dict(meta, passes=SART_PASSES, blocksize=SART_BLOCK, seconds=dt)))
        log(f"os-sart done in {dt:.0f} s")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "both")
