"""Training and evaluation of the learned prior for sparse-view CGLS.

Workload (256^3 volume at 1 mm, 512 x 512 detector at 0.8 mm, 90 views over
the full circle, noiseless data from the same projector that reconstructs):

* training pairs (sparse-view against dense-view reconstructions): for
  phantom seeds s, x_gt = textured random ellipsoids; input = the CGLS
  iterate after k in {5, 10, 15, 20} iterations on the 90 views (the states
  the plug-and-play loop hands the network); target = CGLS after 20
  iterations on 720 views of the same phantom;
* training: random 64^3 crops (batch 4), MSE, Adam (lr 1e-3);
* evaluation: for test seeds, plain CGLS and PnP-CGLS (denoiser every 5
  iterations, accepted when the data residual grows by at most 5 %), PSNR
  over the field-of-view cylinder after every iteration and the solver time
  from GPU events: time to reach 40 dB, and time to reach plain CGLS's best
  PSNR.

Command line (writes JSON / checkpoints where told):
    python -m paper_2412_10129_amd.learned train --phantoms 32 --steps 1500 --out ckpt.pt
    python -m paper_2412_10129_amd.learned evaluate --ckpt ckpt.pt --phantoms 4 --iters 60
    python -m paper_2412_10129_amd.learned bench
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

import synth

from . import algs
from .ops import Plan
from .unet import UNet

KS = (5, 10, 15, 20)


def _phantom(args):
    name, seed = args
    geo, _ = synth.workload(name)
    return synth.textured_phantom(geo, seed)


def phantoms(name: str, seeds: Sequence[int], workers: int = 8) -> List[np.ndarray]:
    """Host phantoms (FP64 voxelisation, FP32 result) in a process pool."""
    workers = max(1, min(workers, len(seeds)))
    if workers == 1:
        return [_phantom((name, s)) for s in seeds]
    with ProcessPoolExecutor(workers) as ex:
        return list(ex.map(_phantom, [(name, s) for s in seeds]))


def data_range(geo, x_gt: np.ndarray) -> float:
    """max - min of the ground truth over the FOV cylinder (the PSNR's R)."""
    nz, ny, nx = geo.nVoxel
    dy, dx = geo.dVoxel[1], geo.dVoxel[2]
    y = (np.arange(ny) + 0.5 - ny / 2) * dy
    x = (np.arange(nx) + 0.5 - nx / 2) * dx
    m = (y[:, None] ** 2 + x[None, :] ** 2) <= geo.iso_fov_radius() ** 2
    vals = x_gt[:, m]
    return float(vals.max() - vals.min())


def make_pairs(plan: Plan, dense: Plan, vols: List[np.ndarray], kind: str = "interp", ks=KS, dense_iters: int = 20):
    """(inputs, targets) on the device: sparse-view CGLS-k iterates and the
    dense-view CGLS reconstruction of the same phantom."""
    inputs, targets = [], []
    for v in vols:
        xg = torch.from_numpy(v).to(plan.device)
        b = plan.forward(xg, kind=kind)
        _, h = algs.cgls(plan, b, max(ks), kind=kind, snapshots=ks, sync=False)
        bd = dense.forward(xg, kind=kind)
        xd, _ = algs.cgls(dense, bd, dense_iters, kind=kind, sync=False)
        del b, bd
        for k in ks:
            inputs.append(h["snapshots"][k])
            targets.append(xd)
    return inputs, targets


def train(net: UNet, inputs, targets, steps: int, crop: int = 64, batch: int = 4, seed: int = 0,
          log_every: int = 100, log=print) -> List[float]:
    """Adam on random crops; returns the per-step MSE (host floats, read
    every `log_every` steps)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    D, H, W = inputs[0].shape
    xb = torch.empty((batch, crop, crop, crop), dtype=torch.float32, device=net.device)
    tb = torch.empty_like(xb)
    sqs = []
    for it in range(steps):
        for j in range(batch):
            i = int(rng.integers(len(inputs)))
            z, y, x = (int(rng.integers(0, n - crop + 1)) for n in (D, H, W))
            xb[j].copy_(inputs[i][z:z + crop, y:y + crop, x:x + crop])
            tb[j].copy_(targets[i][z:z + crop, y:y + crop, x:x + crop])
        sq = net.train_step(xb, tb)
        if (it + 1) % log_every == 0 or it == steps - 1:
            v = float(sq.cpu()) / xb.numel()
            sqs.append(v)
            log(f"step {it + 1}: mse {v:.3e}")
    return sqs


def _first_at(psnr, ms, level):
    t = np.cumsum(ms)
    idx = np.nonzero(np.asarray(psnr) >= level)[0]
    return (float(t[idx[0]]) if len(idx) else None), (int(idx[0]) + 1 if len(idx) else None)


def evaluate(plan: Plan, net: UNet, vols: List[np.ndarray], niter: int = 60, every: int = 5, ratio: float = 1.05,
             kind: str = "interp", target_db: float = 40.0, log=print) -> Dict:
    """Plain CGLS vs PnP-CGLS on each volume: PSNR histories, solver times,
    time to `target_db`, and time for PnP to reach plain CGLS's best."""
    runs = []
    geo = plan.geo
    for n, v in enumerate(vols):
        xg = torch.from_numpy(v).to(plan.device)
        R = data_range(geo, v)
        b = plan.forward(xg, kind=kind)
        res = {}
        for name, ev in (("cgls", niter + 1), ("pnp", every)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, h = algs.pnp_cgls(plan, b, niter, net, every=ev, ratio=ratio, kind=kind, x_gt=xg, data_range=R,
                                 timing=True)
            wall = time.perf_counter() - t0
            res[name] = {"psnr": [float(p) for p in h["psnr"]], "ms": [float(m) for m in h["ms"]],
                         "accepted": h["accepted"], "ratios": h["ratios"], "wall_s": wall}
        best = max(res["cgls"]["psnr"])
        for name in res:
            t, k = _first_at(res[name]["psnr"], res[name]["ms"], target_db)
            res[name]["ms_to_target"], res[name]["iters_to_target"] = t, k
            t, k = _first_at(res[name]["psnr"], res[name]["ms"], best)
            res[name]["ms_to_cgls_best"], res[name]["iters_to_cgls_best"] = t, k
            res[name]["best_psnr"] = max(res[name]["psnr"])
        log(f"volume {n}: cgls best {best:.2f} dB, pnp best {res['pnp']['best_psnr']:.2f} dB; "
            f"to {target_db} dB: cgls {res['cgls']['ms_to_target']} ms, pnp {res['pnp']['ms_to_target']} ms; "
            f"pnp to cgls best {res['pnp']['ms_to_cgls_best']} ms vs {res['cgls']['ms_to_cgls_best']} ms")
        runs.append(res)
    return {"runs": runs, "niter": niter, "every": every, "ratio": ratio, "kind": kind, "target_db": target_db}


def quick_benchmark(train_phantoms: int = 4, steps: int = 600, test_phantoms: int = 2, niter: int = 60,
                    kind: str = "interp", workers: int = 8, log=print) -> Dict:
    """A bounded run of the whole learned-prior pipeline for the benchmark:
    pairs from `train_phantoms` phantoms (seeds 0..), `steps` Adam steps,
    then plain CGLS and PnP-CGLS on `test_phantoms` test volumes (seeds
    10000..).  Returns per-volume times to 40 dB and to plain CGLS's best."""
    t0 = time.perf_counter()
    geo, ang = synth.workload("sparse256")
    plan = Plan(geo, ang)
    dense = Plan(geo, synth.circular_angles(720))
    vols = phantoms("sparse256", range(train_phantoms), workers)
    inputs, targets = make_pairs(plan, dense, vols, kind)
    del dense
    net = UNet(seed=0)
    train(net, inputs, targets, steps, log=lambda m: None)
    del inputs, targets
    test = phantoms("sparse256", range(10000, 10000 + test_phantoms), workers)
    res = evaluate(plan, net, test, niter, kind=kind, log=log)
    rr = res["runs"]
    out = {
        "metric": "time to 40 dB PSNR, PnP-CGLS (learned prior) vs plain CGLS",
        "unit": "ms",
        "config": {"workload": "sparse256", "volume": list(geo.nVoxel), "views": len(ang), "projector": kind,
                   "train_phantoms": train_phantoms, "train_pairs": 4 * train_phantoms, "train_steps": steps,
                   "test_phantoms": test_phantoms, "iterations": niter, "denoise_every": 5},
        "cgls_ms_to_40db": [r["cgls"]["ms_to_target"] for r in rr],
        "pnp_ms_to_40db": [r["pnp"]["ms_to_target"] for r in rr],
        "cgls_best_db": [round(r["cgls"]["best_psnr"], 3) for r in rr],
        "pnp_best_db": [round(r["pnp"]["best_psnr"], 3) for r in rr],
        "cgls_ms_to_cgls_best": [r["cgls"]["ms_to_cgls_best"] for r in rr],
        "pnp_ms_to_cgls_best": [r["pnp"]["ms_to_cgls_best"] for r in rr],
        "wall_s": round(time.perf_counter() - t0, 1),
    }
    return out


def bench_unet(repeat: int = 3, log=print) -> List[Dict]:
    """Forward and training-step times (ms, GPU events) of the U-Net on one
    256^3 volume and on a batch of four 64^3 crops; FLOP/s from the
    network's multiply-adds (3x3x3 and 2x2x2 convolutions, 2 flops each)."""
    net = UNet(seed=0)
    out = []
    for shape in [(1, 256, 256, 256), (4, 64, 64, 64)]:
        x = torch.rand(shape, device=net.device, generator=torch.Generator(device=net.device).manual_seed(0))
        tgt = x * 0.9
        res = {"shape": list(shape)}
        for name, fn in (("fwd_ms", lambda: net.forward(x)), ("train_ms", lambda: net.train_step(x, tgt))):
            fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(repeat):
                fn()
            e1.record()
            torch.cuda.synchronize()
            res[name] = round(e0.elapsed_time(e1) / repeat, 3)
        res["fwd_TFLOP/s"] = round(unet_flops(shape, net.ch) / (res["fwd_ms"] / 1e3) / 1e12, 1)
        log(json.dumps(res))
        out.append(res)
    return out


def unet_flops(shape, channels) -> float:
    """Multiply-add flops of one forward pass (convolutions only)."""
    n, d, h, w = shape
    vox = float(n * d * h * w)
    fl, cin = 0.0, 1            # algorithmic: the first convolution has one input channel
    for lvl, c in enumerate(channels):
        v = vox / 8 ** lvl
        fl += 2 * 27 * v * (cin * c + c * c)
        cin = c
    for lvl in range(len(channels) - 2, -1, -1):
        c, v = channels[lvl], vox / 8 ** lvl
        fl += 2 * v * channels[lvl + 1] * c                 # up-convolution: one tap per output voxel
        fl += 2 * 27 * v * (2 * c * c + c * c)
    return fl


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--phantoms", type=int, default=32)
    t.add_argument("--first-seed", type=int, default=0)
    t.add_argument("--steps", type=int, default=1500)
    t.add_argument("--crop", type=int, default=64)
    t.add_argument("--batch", type=int, default=4)
    t.add_argument("--kind", default="interp")
    t.add_argument("--out", required=True)
    t.add_argument("--workers", type=int, default=8)
    e = sub.add_parser("evaluate")
    e.add_argument("--ckpt", required=True)
    e.add_argument("--phantoms", type=int, default=4)
    e.add_argument("--first-seed", type=int, default=10000)
    e.add_argument("--iters", type=int, default=60)
    e.add_argument("--kind", default="interp")
    e.add_argument("--out", default=None)
    e.add_argument("--workers", type=int, default=8)
    b = sub.add_parser("bench", help="time the U-Net forward and one training step")
    b.add_argument("--repeat", type=int, default=3)
    a = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)
    if a.cmd == "bench":
        bench_unet(a.repeat, log)
        return
    geo, ang = synth.workload("sparse256")
    plan = Plan(geo, ang)
    if a.cmd == "train":
        t0 = time.perf_counter()
        vols = phantoms("sparse256", range(a.first_seed, a.first_seed + a.phantoms), a.workers)
        log(f"{len(vols)} phantoms in {time.perf_counter() - t0:.1f} s")
        t0 = time.perf_counter()
        dense = Plan(geo, synth.circular_angles(720))
        inputs, targets = make_pairs(plan, dense, vols, a.kind)
        del dense
        torch.cuda.synchronize()
        log(f"{len(inputs)} pairs in {time.perf_counter() - t0:.1f} s")
        net = UNet(seed=0)
        t0 = time.perf_counter()
        hist = train(net, inputs, targets, a.steps, a.crop, a.batch, log=log)
        torch.cuda.synchronize()
        log(f"trained {a.steps} steps in {time.perf_counter() - t0:.1f} s")
        torch.save({k: (v.cpu() if isinstance(v, torch.Tensor) else v) for k, v in net.state_dict().items()}, a.out)
        log(json.dumps({"train_mse": hist}))
    else:
        net = UNet(seed=0)
        sd = torch.load(a.ckpt, map_location="cpu", weights_only=True)
        net.load_state_dict({k: (v.to(net.device) if k != "t" else v) for k, v in sd.items()})
        vols = phantoms("sparse256", range(a.first_seed, a.first_seed + a.phantoms), a.workers)
        res = evaluate(plan, net, vols, a.iters, kind=a.kind, log=log)
        summ = {
            "cgls_best_db": [r["cgls"]["best_psnr"] for r in res["runs"]],
            "pnp_best_db": [r["pnp"]["best_psnr"] for r in res["runs"]],
            "cgls_ms_to_40db": [r["cgls"]["ms_to_target"] for r in res["runs"]],
            "pnp_ms_to_40db": [r["pnp"]["ms_to_target"] for r in res["runs"]],
            "cgls_ms_to_cgls_best": [r["cgls"]["ms_to_cgls_best"] for r in res["runs"]],
            "pnp_ms_to_cgls_best": [r["pnp"]["ms_to_cgls_best"] for r in res["runs"]],
        }
        log(json.dumps(summ))
        if a.out:
            with open(a.out, "w") as f:
                json.dump({"summary": summ, **res}, f)


if __name__ == "__main__":
    main()
