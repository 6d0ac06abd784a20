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

Pairs are numbered: with the input iterations ks (KS by default, KS8 for
the full training set), pair p comes from phantom seed p // len(ks) with
the input after k = ks[p % len(ks)] iterations, so phantoms 0..249 give
pairs 0..1999 with KS8.
Training can run in segments: each `train` call makes the pairs of its own
phantom range, trains on them, and saves the network with its Adam state;
the next call resumes from that checkpoint with the next range (the pairs
stream through the training once, a segment at a time).

Command line (writes JSON / checkpoints where told):
    python -m paper_2412_10129_amd.learned train --phantoms 32 --steps 1500 --out ckpt.pt
    python -m paper_2412_10129_amd.learned train --first-seed 32 --phantoms 32 --resume ckpt.pt --out ckpt2.pt
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
KS8 = (3, 5, 8, 10, 13, 15, 18, 20)


def _phantom(args):
    name, seed = args
    geo, _ = synth.workload(name)
    return synth.textured_phantom(geo, seed)


def phantoms(name: str, seeds: Sequence[int], workers: int = 8) -> List[np.ndarray]:
    """Host phantoms (FP64 voxelisation, FP32 result) in a process pool."""
    return list(phantom_stream(name, seeds, workers))


def phantom_stream(name: str, seeds: Sequence[int], workers: int = 8):
    """The same phantoms, yielded in seed order as the pool finishes them,
    so the GPU can work on the first ones while the host makes the rest."""
    workers = max(1, min(workers, len(seeds)))
    if workers == 1:
        for s in seeds:
            yield _phantom((name, s))
        return
    with ProcessPoolExecutor(workers) as ex:
        futs = [ex.submit(_phantom, (name, s)) for s in seeds]
        for f in futs:
            yield f.result()


def data_range(geo, x_gt: np.ndarray) -> float:
    """max - min of the ground truth over the FOV cylinder (the PSNR's R)."""
    nz, ny, nx = geo.nVoxel
    dy, dx = geo.dVoxel[1], geo.dVoxel[2]
    y = (np.arange(ny) + 0.5 - ny / 2) * dy
    x = (np.arange(nx) + 0.5 - nx / 2) * dx
    m = (y[:, None] ** 2 + x[None, :] ** 2) <= geo.iso_fov_radius() ** 2
    vals = x_gt[:, m]
    return float(vals.max() - vals.min())


def make_pairs(plan: Plan, dense: Plan, vols, kind: str = "interp", ks=KS, dense_iters: int = 20, log=None,
               log_every: int = 5):
    """(inputs, targets) on the device: sparse-view CGLS-k iterates and the
    dense-view CGLS reconstruction of the same phantom (`vols` may be any
    iterable of host phantoms).  With `log`, a progress line every
    `log_every` phantoms (after the device has finished them)."""
    inputs, targets = [], []
    t0 = time.perf_counter()
    for n, v in enumerate(vols):
        if log is not None and n and n % log_every == 0:
            torch.cuda.synchronize()
            log(f"pairs of {n} phantoms in {time.perf_counter() - t0:.1f} s")
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
          log_every: int = 100, log=print, rng: Optional[np.random.Generator] = None) -> List[float]:
    """Adam on random crops; returns the per-step MSE (host floats, read
    every `log_every` steps).  Crops are drawn from `rng` (advanced in
    place) if given, else from a PCG64 stream seeded with `seed`."""
    rng = np.random.Generator(np.random.PCG64(seed)) if rng is None else rng
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


def evaluate(plan: Plan, net: UNet, vols, niter: int = 60, every: int = 5, ratio: float = 1.05,
             kind: str = "interp", target_db: float = 40.0, log=print, on_run=None) -> Dict:
    """Plain CGLS vs PnP-CGLS on each volume: PSNR histories, solver times,
    time to `target_db`, and time for PnP to reach plain CGLS's best.

    With `on_run`, every iterate of both runs is kept on the device and
    on_run(n, x_gt_host, res, iterates) is called per volume with
    iterates = {"cgls": [...], "pnp": [...]} (device tensors, freed after
    the call), e.g. to score them independently."""
    runs = []
    geo = plan.geo
    for n, v in enumerate(vols):
        xg = torch.from_numpy(v).to(plan.device)
        R = data_range(geo, v)
        b = plan.forward(xg, kind=kind)
        res = {}
        its = {}
        for name, ev in (("cgls", niter + 1), ("pnp", every)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            its[name] = [] if on_run is not None else None
            _, h = algs.pnp_cgls(plan, b, niter, net, every=ev, ratio=ratio, kind=kind, x_gt=xg, data_range=R,
                                 timing=True, keep=its[name])
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
        if on_run is not None:
            on_run(n, v, res, its)
        del its
        runs.append(res)
    return {"runs": runs, "niter": niter, "every": every, "ratio": ratio, "kind": kind, "target_db": target_db}


WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "unet_sparse256.pt")


def training_checkpoint(net: UNet, rng: np.random.Generator) -> Dict:
    """Everything a training run resumes from: the FP32 parameters, the Adam
    moments and step, and the crop sampler's generator state (as JSON), all
    on the host (torch.save it; the safe loader reads it back)."""
    sd = {k: (v.detach().cpu() if isinstance(v, torch.Tensor) else v) for k, v in net.state_dict().items()}
    sd["rng"] = json.dumps(rng.bit_generator.state)
    return sd


def restore_training(net: UNet, sd: Dict) -> np.random.Generator:
    """Load a training_checkpoint into `net`; returns the crop sampler at the
    state it was saved in, so that training continues bit for bit."""
    net.load_state_dict({k: sd[k] for k in ("params", "m", "v", "t")})
    rng = np.random.Generator(np.random.PCG64())
    rng.bit_generator.state = json.loads(sd["rng"])
    return rng


def save_weights(params: torch.Tensor, path: str, meta: Dict) -> None:
    """A trained network's FP32 parameters (no optimiser state) with a
    description of its training."""
    torch.save({"params": params.detach().cpu().contiguous(), "meta": json.dumps(meta)}, path)


def load_weights(net: UNet, path: str) -> Dict:
    sd = torch.load(path, map_location="cpu", weights_only=True)
    net.params.copy_(sd["params"].to(net.device))
    net.pack()
    return json.loads(sd["meta"])


def quick_benchmark(train_phantoms: int = 4, steps: int = 600, test_phantoms: int = 2, niter: int = 60,
                    kind: str = "interp", workers: int = 8, log=print, weights: Optional[str] = None) -> Dict:
    """A bounded run of the learned prior for the benchmark: with `weights`
    (a saved trained network) plain CGLS and PnP-CGLS with that network on
    `test_phantoms` test volumes (seeds 10000..); otherwise first a short
    training run (pairs from `train_phantoms` phantoms, seeds 0.., `steps`
    Adam steps).  Returns per-volume times to 40 dB and to plain CGLS's
    best."""
    t0 = time.perf_counter()
    geo, ang = synth.workload("sparse256")
    plan = Plan(geo, ang)
    net = UNet(seed=0)
    trained = None
    if weights and os.path.exists(weights):
        trained = load_weights(net, weights)
    else:
        dense = Plan(geo, synth.circular_angles(720))
        vols = phantoms("sparse256", range(train_phantoms), workers)
        inputs, targets = make_pairs(plan, dense, vols, kind)
        del dense
        train(net, inputs, targets, steps, log=lambda m: None)
        del inputs, targets
    test = phantoms("sparse256", range(10000, 10000 + test_phantoms), workers)
    res = evaluate(plan, net, test, niter, kind=kind, log=log)
    rr = res["runs"]
    out = {
        "metric": "time to 40 dB PSNR, PnP-CGLS (learned prior) vs plain CGLS",
        "unit": "ms",
        "config": ({"workload": "sparse256", "volume": list(geo.nVoxel), "views": len(ang), "projector": kind,
                    "network": "saved weights", "training": trained, "test_phantoms": test_phantoms,
                    "iterations": niter, "denoise_every": 5} if trained is not None else
                   {"workload": "sparse256", "volume": list(geo.nVoxel), "views": len(ang), "projector": kind,
                    "network": "trained in the run (reduced)", "train_phantoms": train_phantoms,
                    "train_pairs": len(KS) * train_phantoms, "train_steps": steps, "test_phantoms": test_phantoms,
                    "iterations": niter, "denoise_every": 5}),
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
    t.add_argument("--resume", default=None, help="checkpoint (network and Adam state) to continue from")
    t.add_argument("--seed", type=int, default=0, help="crop sampling seed of this segment")
    t.add_argument("--ks", default=",".join(map(str, KS)), help="CGLS iterations of the inputs, e.g. 3,5,8,10,13,15,18,20")
    e = sub.add_parser("evaluate")
    e.add_argument("--ckpt", required=True)
    e.add_argument("--phantoms", type=int, default=4)
    e.add_argument("--first-seed", type=int, default=10000)
    e.add_argument("--iters", type=int, default=60)
    e.add_argument("--kind", default="interp")
    e.add_argument("--out", default=None)
    e.add_argument("--workers", type=int, default=8)
    x = sub.add_parser("export", help="save a checkpoint's network parameters as the weights file")
    x.add_argument("--ckpt", required=True)
    x.add_argument("--out", default=WEIGHTS)
    x.add_argument("--pairs", type=int, required=True)
    x.add_argument("--ks", default=",".join(map(str, KS8)))
    b = sub.add_parser("bench", help="time the U-Net forward and one training step")
    b.add_argument("--repeat", type=int, default=3)
    a = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)
    if a.cmd == "bench":
        bench_unet(a.repeat, log)
        return
    if a.cmd == "export":
        # a checkpoint holds the FP32 master parameters with the Adam state;
        # the weights file keeps the parameters only (no GPU needed)
        sd = torch.load(a.ckpt, map_location="cpu", weights_only=True)
        seen = sorted(int(v) for v in sd.get("phantoms", torch.zeros(0, dtype=torch.int64)).tolist())
        meta = {"pairs": a.pairs, "phantom_seeds": [seen[0], seen[-1]] if seen else None, "phantoms": len(seen),
                "input_iterations": a.ks, "target": "CGLS-20 on 720 views", "adam_steps": int(sd["t"]),
                "crop": 64, "batch": 4}
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        save_weights(sd["params"], a.out, meta)
        log(json.dumps(meta))
        return
    geo, ang = synth.workload("sparse256")
    plan = Plan(geo, ang)
    if a.cmd == "train":
        t0 = time.perf_counter()
        seeds = range(a.first_seed, a.first_seed + a.phantoms)
        dense = Plan(geo, synth.circular_angles(720))
        ks = tuple(int(k) for k in a.ks.split(","))
        inputs, targets = make_pairs(plan, dense, phantom_stream("sparse256", seeds, a.workers), a.kind, ks=ks,
                                     log=log)
        del dense
        torch.cuda.synchronize()
        nk = len(ks)
        log(f"pairs {nk * a.first_seed}..{nk * (a.first_seed + a.phantoms) - 1} ({len(inputs)}, inputs after "
            f"{a.ks} iterations) from phantoms {a.first_seed}..{a.first_seed + a.phantoms - 1} in "
            f"{time.perf_counter() - t0:.1f} s")
        net = UNet(seed=0)
        seen = []
        if a.resume:
            sd = torch.load(a.resume, map_location="cpu", weights_only=True)
            net.load_state_dict({k: (v.to(net.device) if k != "t" else v) for k, v in sd.items()
                                 if k in ("params", "m", "v", "t")})
            seen = [int(v) for v in sd.get("phantoms", torch.zeros(0, dtype=torch.int64)).tolist()]
            log(f"resumed at Adam step {net.t} ({len(seen)} phantoms seen)")
        t0 = time.perf_counter()
        hist = train(net, inputs, targets, a.steps, a.crop, a.batch, seed=a.seed, log=log)
        torch.cuda.synchronize()
        log(f"trained {a.steps} steps in {time.perf_counter() - t0:.1f} s")
        sd = {k: (v.cpu() if isinstance(v, torch.Tensor) else v) for k, v in net.state_dict().items()}
        sd["phantoms"] = torch.tensor(seen + list(seeds), dtype=torch.int64)
        torch.save(sd, a.out)
        log(json.dumps({"train_mse": hist}))
    else:
        net = UNet(seed=0)
        sd = torch.load(a.ckpt, map_location="cpu", weights_only=True)
        net.load_state_dict({k: (v.to(net.device) if k != "t" else v) for k, v in sd.items()
                             if k in ("params", "m", "v", "t")})
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
