"""Time to 40 dB of PnP-CGLS (the learned prior) against plain CGLS on the
sparse-view 256^3 workload, with every PSNR that decides a time re-judged by
the FP64 oracle on the saved iterates (test infrastructure: the solvers run
through the HIP library; only the judging here uses the oracle).

For each test phantom (seeds from --first-seed), both solvers run --iters
iterations with every iterate kept on the GPU.  The device PSNR history
(FP64 sums on the GPU) proposes where a run first reaches a level; the
oracle's PSNR (x_gt = the phantom, over the FOV cylinder, FP64 on the host)
is then evaluated on the iterates around that point and the crossing is the
first iterate the oracle puts at or above the level, with the one before it
below.  Levels: 40 dB, and plain CGLS's best PSNR (oracle value of its best
iterate).  Times are the solver's GPU-event times summed up to the crossing.

    python tests/score_learned.py --ckpt CKPT --phantoms 20 --out result.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def crossing(level, dev_psnr, score):
    """First iterate index whose oracle PSNR is >= level (None if none):
    starts from the device's proposal and walks until the oracle agrees
    that the iterate before is below the level."""
    dev = np.asarray(dev_psnr)
    idx = np.nonzero(dev >= level - 0.05)[0]
    if len(idx) == 0:
        return None
    k = int(idx[0])
    while k < len(dev) and score(k) < level:
        k += 1
    if k == len(dev):
        return None
    while k > 0 and score(k - 1) >= level:
        k -= 1
    return k


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--ckpt", required=True)
    ap.add_argument("--phantoms", type=int, default=20)
    ap.add_argument("--first-seed", type=int, default=10000)
    ap.add_argument("--iters", type=int, default=60)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)

    import torch

    import oracle
    import synth
    from paper_2412_10129_amd import learned as LN
    from paper_2412_10129_amd.ops import Plan
    from paper_2412_10129_amd.unet import UNet

    geo, ang = synth.workload("sparse256")
    plan = Plan(geo, ang)
    net = UNet(seed=0)
    sd = torch.load(a.ckpt, map_location="cpu", weights_only=True)
    net.load_state_dict({k: (v.to(net.device) if k != "t" else v) for k, v in sd.items()
                         if k in ("params", "m", "v", "t")})
    mask = oracle.fov_mask(geo)
    out = {"ckpt_phantoms": len(sd.get("phantoms", [])), "adam_steps": int(net.t), "iters": a.iters,
           "first_seed": a.first_seed, "volumes": []}
    log = lambda m: print(m, flush=True)

    def on_run(n, x_gt, res, its):
        cache = {}

        def score_fn(name):
            def score(k):
                if (name, k) not in cache:
                    cache[(name, k)] = oracle.psnr(its[name][k].cpu().numpy(), x_gt, mask)
                return cache[(name, k)]
            return score
        rec = {"seed": a.first_seed + n}
        jc, jp = score_fn("cgls"), score_fn("pnp")
        kbest = int(np.argmax(res["cgls"]["psnr"]))
        best = jc(kbest)
        rec["cgls_best_db_oracle"] = best
        rec["cgls_best_iter"] = kbest + 1
        for name, score in (("cgls", jc), ("pnp", jp)):
            ms = np.cumsum(res[name]["ms"])
            k40 = crossing(40.0, res[name]["psnr"], score)
            kb = crossing(best, res[name]["psnr"], score)
            rec[name] = {"iters_to_40db": None if k40 is None else k40 + 1,
                         "ms_to_40db": None if k40 is None else float(ms[k40]),
                         "iters_to_cgls_best": None if kb is None else kb + 1,
                         "ms_to_cgls_best": None if kb is None else float(ms[kb]),
                         "best_db_device": float(max(res[name]["psnr"])),
                         "ms_per_iter": float(np.mean(res[name]["ms"])),
                         "accepted": res[name]["accepted"]}
        rec["oracle_judged"] = {f"{nm}@{k + 1}": round(v, 4) for (nm, k), v in sorted(cache.items())}
        dev = {f"{nm}@{k + 1}": round(float(res[nm]["psnr"][k]), 4) for (nm, k) in sorted(cache)}
        rec["max_abs_device_minus_oracle_db"] = max(abs(dev[key] - rec["oracle_judged"][key]) for key in dev)
        log(json.dumps(rec))
        out["volumes"].append(rec)

    t0 = time.perf_counter()
    LN.evaluate(plan, net, LN.phantom_stream("sparse256", range(a.first_seed, a.first_seed + a.phantoms), a.workers),
                a.iters, log=log, on_run=on_run)
    vols = out["volumes"]
    reach = lambda nm: [v[nm]["ms_to_40db"] for v in vols]
    both = [(v["cgls"]["ms_to_40db"], v["pnp"]["ms_to_40db"]) for v in vols
            if v["cgls"]["ms_to_40db"] is not None and v["pnp"]["ms_to_40db"] is not None]
    best_sp = [v["cgls"]["ms_to_cgls_best"] / v["pnp"]["ms_to_cgls_best"] for v in vols
               if v["pnp"]["ms_to_cgls_best"] is not None]
    out["summary"] = {
        "volumes": len(vols),
        "cgls_reached_40db": sum(t is not None for t in reach("cgls")),
        "pnp_reached_40db": sum(t is not None for t in reach("pnp")),
        "median_speedup_to_40db_where_both": float(np.median([c / p for c, p in both])) if both else None,
        "median_speedup_to_cgls_best": float(np.median(best_sp)) if best_sp else None,
        "pnp_reached_cgls_best": len(best_sp),
        "wall_s": round(time.perf_counter() - t0, 1),
    }
    log(json.dumps(out["summary"]))
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
