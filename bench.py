"""Benchmark of the cone-beam projector hot path on one MI355X.

A step is one CGLS iteration on the 512^3 x 720-view workload (1024x768
detector): q = A p, |q|^2, x/r update with |r|^2, s = A^T r, |s|^2, p update
-- the forward projector, its exact transpose and the vector updates, with
every input resident in HBM.  The reported value is A and A^T voxel-view
updates per second: 2 * N^3 * views / step time.

After the timed steps each operator (Siddon A and A^T, interpolated A and
A^T, FDK filter, FDK backprojector) is timed on its own for the breakdown,
a bounded learned-prior run measures the metric's second half (time to
40 dB of PnP-CGLS with the U-Net against plain CGLS, sparse-view 256^3), and
the FP64 CPU oracle is timed on a one-view sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--projector interp|siddon]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# published MI355X peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_VECTOR_TFLOPS = 157.3

# algorithmic FP32 flops per unit of work (add/mul/sub/floor = 1, fma = 2):
#   interpolated A, per sample: position 3 fma (6), floor 3, fraction 3,
#     1 - f 3, seven lerps (mul + fma = 3 each) 21, accumulate 1      = 37
#   interpolated A^T, per sample: position 6, floor 3, fraction 3, 1 - f 3,
#     eight corner weights (2 mul each) 16, times y 8, accumulate 8    = 47
#   Siddon A, per segment: 3-way min 2, clip min 1, length sub 1,
#     accumulate fma 2, exit compare 1, next plane add 1 + fma 2       = 10
#   Siddon A^T, per segment: the same with one multiply by y           = 11
#   FDK backprojection, per voxel-view update: v position fma 2, floor 1,
#     fraction 1, 1 - f 1, two u-lerps 6, v-lerp 3, weight fma 2       = 16
FLOPS = {"interp_fwd": 37, "interp_bwd": 47, "siddon_fwd": 10, "siddon_bwd": 11, "fdk_bp": 16}

# source file of each timed kernel (the HBM traffic recorded for a kernel in
# profiles/traffic.json is used only while that file is unchanged)
KERNEL_SOURCE = {"interp_fwd": "forward.hip", "siddon_fwd": "forward.hip", "interp_bwd": "backward.hip",
                 "siddon_bwd": "backward.hip", "fdk_bp": "fdk.hip"}


def _sha256(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs recorded in profiles/traffic.json, scaled by the plain-copy
    calibration stored there; None if absent or if the kernel's source has
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    k = rec.get("kernels", {}).get(kernel)
    src = os.path.join(ROOT, "paper_2412_10129_amd", "csrc", KERNEL_SOURCE[kernel])
    if not k or not os.path.exists(src) or k.get("source_sha256") != _sha256(src):
        return None
    cal = rec["calibration"]
    return int(1024 * (k["fetch_kib"] * cal["fetch_factor"] + k["write_kib"] * cal["write_factor"]))


def profile_summary(db_path, top=12):
    """Markdown tables of a rocprofv3 results database: kernel durations
    (kernel trace) and per-dispatch averages of any PMC counters."""
    import collections
    import re
    import sqlite3
    con = sqlite3.connect(db_path)
    short = lambda n: re.sub(r"^void ", "", n.replace("ctmi::(anonymous namespace)::", "").split("(")[0]).strip()
    lines = []
    tables = {r[0] for r in con.execute("select name from sqlite_master where type in ('table', 'view')")}
    if "top_kernels" in tables:
        rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
        if rows:
            lines += ["| kernel | calls | avg (ms) | total (ms) | % |", "|---|---|---|---|---|"]
            for name, calls, tot, avg, pct in rows[:top]:
                lines.append(f"| {short(name)} | {calls} | {avg / 1e3:.3f} | {tot / 1e3:.3f} | {pct:.2f} |")
    if "pmc_events" in tables:
        rows = con.execute("select name, dispatch_id, counter_name, sum(counter_value) from pmc_events "
                           "group by name, dispatch_id, counter_name").fetchall()
        acc = collections.defaultdict(lambda: collections.defaultdict(list))
        for name, _, cn, v in rows:
            acc[short(name)][cn].append(v)
        if acc:
            cnames = sorted({c for d in acc.values() for c in d})
            lines += ["", "| kernel | dispatches | " + " | ".join(f"{c} (avg/dispatch)" for c in cnames) + " |",
                      "|---|---|" + "---|" * len(cnames)]
            for k, d in sorted(acc.items()):
                nd = max(len(v) for v in d.values())
                vals = " | ".join(f"{sum(d[c]) / len(d[c]):.6g}" if c in d else "" for c in cnames)
                lines.append(f"| {k} | {nd} | {vals} |")
    return "\n".join(lines)


def _rays(geo, angles):
    """Ray end points in voxel-cell coordinates for the listed views (FP64)."""
    nz, ny, nx = geo.nVoxel
    dz, dy, dx = geo.dVoxel
    oz, oy, ox = geo.offOrigin
    lo = np.array([ox - nx * dx / 2, oy - ny * dy / 2, oz - nz * dz / 2])
    h = np.array([dx, dy, dz])
    nv, nu = geo.nDetector
    iv, iu = np.meshgrid(np.arange(nv), np.arange(nu), indexing="ij")
    u = (iu + 0.5 - nu / 2) * geo.dDetector[1] + geo.offDetector[1]
    v = (iv + 0.5 - nv / 2) * geo.dDetector[0] + geo.offDetector[0]
    for th in angles:
        c, s = math.cos(th), math.sin(th)
        S = np.array([geo.DSO * c, geo.DSO * s, 0.0])
        P = np.stack([S[0] - geo.DSD * c - u * s, S[1] - geo.DSD * s + u * c, v], -1).reshape(-1, 3)
        yield (S - lo) / h, (P - lo) / h, h


def work_units(geo, nviews, sample_views=16):
    """Interpolation samples and Siddon segments of all rays, counted
    exactly on `sample_views` evenly spaced views and scaled to all views
    (work is uniform over the views of a circular orbit)."""
    n = np.array([geo.nVoxel[2], geo.nVoxel[1], geo.nVoxel[0]], dtype=np.float64)
    ds = geo.accuracy * min(geo.dVoxel)
    ang = 2 * np.pi * np.arange(sample_views) / sample_views
    samples = segments = 0.0
    for Sc, P, h in _rays(geo, ang):
        D = P - Sc
        L = np.linalg.norm(D * h, axis=1)
        # samples: open box (-1, n) in voxel-centre coordinates, t = k ds
        st = D * (ds / L)[:, None]
        with np.errstate(divide="ignore", invalid="ignore"):
            ka = (-1.0 - (Sc - 0.5)) / st
            kb = (n - (Sc - 0.5)) / st
        kmin = np.maximum(np.nanmax(np.minimum(ka, kb), 1), 0.0)
        kmax = np.minimum(np.nanmin(np.maximum(ka, kb), 1), L / ds)
        cnt = np.floor(kmax) - np.ceil(kmin) + 1
        samples += float(np.sum(np.where(kmax > kmin, np.maximum(cnt, 0), 0)))
        # segments: cells visited = 1 + planes crossed between entry and exit
        with np.errstate(divide="ignore", invalid="ignore"):
            a0 = (0.0 - Sc) / D
            a1 = (n - Sc) / D
        amin = np.maximum(np.nanmax(np.minimum(a0, a1), 1), 0.0)
        amax = np.minimum(np.nanmin(np.maximum(a0, a1), 1), 1.0)
        hit = amax > amin
        e = Sc + amin[:, None] * D
        x = Sc + amax[:, None] * D
        cross = np.sum(np.abs(np.floor(np.clip(x, 0, n - 1e-9)) - np.floor(np.clip(e, 0, n - 1e-9))), 1)
        segments += float(np.sum(np.where(hit, cross + 1, 0)))
    scale = nviews / sample_views
    return samples * scale, segments * scale


def cpu_baseline(geo, angles, x, y, kind):
    """The FP64 oracle on one view of the workload: forward and backward."""
    import oracle
    oracle._L()
    a1 = angles[:1]
    x64 = x.astype(np.float64)
    t0 = time.perf_counter()
    oracle.forward(geo, a1, x64, kind)
    t1 = time.perf_counter()
    oracle.backward(geo, a1, y[:1].astype(np.float64), kind)
    t2 = time.perf_counter()
    upd = float(np.prod(geo.nVoxel))
    return {"value": 2 * upd / (t2 - t0), "unit": "voxel-view updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"FP64 {kind} A and A^T, 1 of {len(angles)} views of the 512^3 workload "
                      f"(A {t1 - t0:.1f} s, A^T {t2 - t1:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cbct512")
    ap.add_argument("--projector", default="interp", choices=["interp", "siddon"])
    ap.add_argument("--no-breakdown", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-prior run (training pairs, training, PnP-CGLS vs CGLS)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (reference for HBM byte counters)")
    ap.add_argument("--profile-summary", metavar="DB",
                    help="only print markdown tables of a rocprofv3 results database and exit")
    ap.add_argument("--top", type=int, default=12, help="kernels listed by --profile-summary")
    args = ap.parse_args()
    if args.profile_summary:
        print(profile_summary(args.profile_summary, top=args.top))
        return
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        c = torch.empty_like(a)
        c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": c.numel() * 4}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the view-sharded multi-GPU "
              "layout is a design only in this repository)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2412_10129_amd as P
    import synth

    geo, angles = synth.workload(args.workload)
    nviews = len(angles)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print(f"[bench] workload {args.workload}: vol {geo.nVoxel} det {geo.nDetector} views {nviews}", flush=True)
    x_h = synth.uniform_volume(geo, 4)
    y_h = synth.uniform_projections(geo, nviews, 5)
    plan = P.Plan(geo, angles, dev)
    kind = args.projector
    x = torch.from_numpy(x_h).to(dev)
    b = torch.from_numpy(y_h).to(dev)
    # CGLS state (Hestenes-Stiefel): x = 0, r = b, s = A^T b, p = s,
    # gamma_0 = |s|^2; the scalars live on the device in two rotating rows
    # [gamma, delta, |r|^2, spare] so every step is a true CGLS iteration.
    from paper_2412_10129_amd import ops
    xs = torch.zeros_like(x)
    r = b.clone()
    s = plan.backproject(r, kind=kind)
    p = s.clone()
    q = torch.empty_like(b)
    ws = ops._ws(dev)
    sc = torch.zeros((2, 4), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def slot(row, col):
        return sc.data_ptr() + 8 * (4 * row + col)

    def dot_into(u, addr):
        ops.L.check(ops.L.lib().ctmi_dot(ops._ptr(u, "u"), ops._ptr(u, "u"), u.numel(), addr, ws.data_ptr(),
                                         ws.numel() * 8, ops._stream()))

    dot_into(s, slot(0, 0))
    ev_f0, ev_f1, ev_b0, ev_b1 = [], [], [], []
    it = [0]

    def step(record=False):
        cur = it[0] % 2
        nxt = 1 - cur
        if record:
            e = torch.cuda.Event(enable_timing=True); e.record(stream); ev_f0.append(e)
        plan.forward(p, out=q, kind=kind)
        if record:
            e = torch.cuda.Event(enable_timing=True); e.record(stream); ev_f1.append(e)
        dot_into(q, slot(cur, 1))
        ops.cgls_xr(xs, p, r, q, slot(cur, 0), slot(cur, 1), slot(cur, 2), ws)
        if record:
            e = torch.cuda.Event(enable_timing=True); e.record(stream); ev_b0.append(e)
        plan.backproject(r, out=s, kind=kind)
        if record:
            e = torch.cuda.Event(enable_timing=True); e.record(stream); ev_b1.append(e)
        dot_into(s, slot(nxt, 0))
        ops.cgls_p(p, s, slot(cur, 0), slot(nxt, 0))
        it[0] += 1

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps)", flush=True)
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        step(record=True)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the iterate must stay finite (a diverged state would let kernels skip work)
    h = sc.cpu().numpy()
    if not (np.all(np.isfinite(h)) and bool(torch.isfinite(xs).all()) and bool(torch.isfinite(r).all())):
        raise RuntimeError(f"CGLS state is not finite after the timed steps: {h}")
    ms = e0.elapsed_time(e1) / args.steps
    t_fwd = np.mean([a_.elapsed_time(b_) for a_, b_ in zip(ev_f0, ev_f1)])
    t_bwd = np.mean([a_.elapsed_time(b_) for a_, b_ in zip(ev_b0, ev_b1)])
    upd = float(np.prod(geo.nVoxel)) * nviews
    value = 2 * upd / (ms / 1e3)
    print(f"[bench] {args.steps} steps: {ms:.2f} ms/step (wall {wall:.2f} s); A {t_fwd:.2f} ms, A^T {t_bwd:.2f} ms; "
          f"|r|^2 {h[0, 2]:.6g} / {h[1, 2]:.6g}", flush=True)

    samples, segments = work_units(geo, nviews)
    units = {"interp_fwd": samples, "interp_bwd": samples, "siddon_fwd": segments, "siddon_bwd": segments}
    kf, kb = f"{kind}_fwd", f"{kind}_bwd"
    dominant, t_dom = (kb, t_bwd) if t_bwd >= t_fwd else (kf, t_fwd)
    fl = FLOPS[dominant] * units[dominant]
    ach = fl / (t_dom / 1e3) / 1e12
    roofline = {"bound": "alu", "kernel": dominant, "achieved": round(ach, 3), "peak": PEAK_FP32_VECTOR_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_VECTOR_TFLOPS, 4),
                "traffic": recorded_traffic(dominant),
                "work_units": units[dominant], "flops_per_unit": FLOPS[dominant],
                "avg_launch_ms": round(float(t_dom), 3)}

    breakdown = {}
    if not args.no_breakdown:
        fl_fdk = float(np.prod(geo.nVoxel)) * nviews
        ops_list = [
            ("siddon_fwd", lambda: plan.forward(x, out=q, kind="siddon")),
            ("siddon_bwd", lambda: plan.backproject(b, out=s, kind="siddon")),
            ("interp_fwd", lambda: plan.forward(x, out=q, kind="interp")),
            ("interp_bwd", lambda: plan.backproject(b, out=s, kind="interp")),
            ("fdk_filter", lambda: plan.fdk_filter(b, out=q)),
            ("fdk_bp", lambda: plan.backproject(b, out=s, kind="fdk")),
        ]
        for name, fn in ops_list:
            fn()
            ea = torch.cuda.Event(enable_timing=True)
            eb = torch.cuda.Event(enable_timing=True)
            ea.record(stream)
            for _ in range(2):
                fn()
            eb.record(stream)
            torch.cuda.synchronize()
            t = ea.elapsed_time(eb) / 2
            ent = {"ms": round(t, 3)}
            if name == "fdk_filter":
                ent["GB/s"] = round(2 * 4 * b.numel() / (t / 1e3) / 1e9, 1)
            else:
                ent["updates/s"] = float(f"{upd / (t / 1e3):.4g}")
                u = units.get(name, fl_fdk)
                ent["TFLOP/s"] = round(FLOPS[name] * u / (t / 1e3) / 1e12, 3)
            breakdown[name] = ent
            print(f"[bench] {name}: {ent}", flush=True)

        # the wider solver rows at the same size: elementwise and stencil
        # kernels against their algorithmic HBM bytes, one MLEM iteration and
        # one OS-ASD-POCS iteration (blocks of 20 views, 20 AwTV steps)
        from paper_2412_10129_amd import ops as O
        from paper_2412_10129_amd import algs as AL
        nvox = x.numel()
        xs = x.clone()
        bps = s.clone()
        gn = O.dot(s, s)
        extra = [
            ("awtv_grad", lambda: O.awtv_grad(x, out=s, delta=0.5), 8.0 * nvox),
            ("tv_step", lambda: O.tv_step(xs, s, gn, 1e-3), 12.0 * nvox),
            ("em_ratio", lambda: O.em_ratio(b, q, q), 12.0 * b.numel()),
            ("em_update", lambda: O.em_update(xs, bps, bps), 16.0 * nvox),
        ]
        for name, fn, nbytes in extra:
            fn()
            ea = torch.cuda.Event(enable_timing=True)
            eb = torch.cuda.Event(enable_timing=True)
            ea.record(stream)
            for _ in range(3):
                fn()
            eb.record(stream)
            torch.cuda.synchronize()
            t = ea.elapsed_time(eb) / 3
            ent = {"ms": round(t, 3), "GB/s": round(nbytes / (t / 1e3) / 1e9, 1),
                   "frac_hbm": round(nbytes / (t / 1e3) / 8e12, 3)}
            breakdown[name] = ent
            print(f"[bench] {name}: {ent}", flush=True)
        del xs, bps
        # the projectors under per-view geometry at the same size: orbit
        # tilted by 0.2 rad, 1.5 mm centre-of-rotation shift, detector turned
        # by (0.02, 0.01, -0.015) rad
        import types
        ang = np.asarray(plan.angles, dtype=np.float64)
        nv_ = len(ang)
        gviews = types.SimpleNamespace(
            angles=np.stack([ang, np.full(nv_, 0.2), np.zeros(nv_)], axis=1), DSO=np.full(nv_, geo.DSO),
            DSD=np.full(nv_, geo.DSD), offOrigin=np.zeros((nv_, 3)), offDetector=np.zeros((nv_, 2)),
            COR=np.full(nv_, 1.5), rotDetector=np.tile([0.02, 0.01, -0.015], (nv_, 1)))
        gplan = P.Plan(geo, gviews, dev)
        for name, fn in (("interp_fwd_general", lambda: gplan.forward(x, out=q, kind="interp")),
                         ("interp_bwd_general", lambda: gplan.backproject(b, out=s, kind="interp"))):
            fn()
            ea = torch.cuda.Event(enable_timing=True)
            eb = torch.cuda.Event(enable_timing=True)
            ea.record(stream)
            fn()
            eb.record(stream)
            torch.cuda.synchronize()
            t = ea.elapsed_time(eb)
            breakdown[name] = {"ms": round(t, 3), "updates/s": float(f"{upd / (t / 1e3):.4g}")}
            print(f"[bench] {name}: {breakdown[name]}", flush=True)
        del gplan
        for name, make, it in (("mlem_iter", lambda: AL.OSEM(plan, None, kind), None),
                               ("os_asd_pocs_iter", lambda: AL.ASDPOCS(plan, 20, kind), None)):
            solver = make()
            torch.cuda.synchronize()
            ea = torch.cuda.Event(enable_timing=True)
            eb = torch.cuda.Event(enable_timing=True)
            ea.record(stream)
            if name == "mlem_iter":
                xm = torch.ones_like(x)
                solver.step(xm, b)
            else:
                solver.run(b, 1)
            eb.record(stream)
            torch.cuda.synchronize()
            t = ea.elapsed_time(eb)
            breakdown[name] = {"ms": round(t, 1), "updates/s": float(f"{2 * upd / (t / 1e3):.4g}")}
            print(f"[bench] {name}: {breakdown[name]}", flush=True)
            del solver

    learned = None
    if not args.no_learned:
        # the second half of the headline metric: time to 40 dB of the learned
        # prior inside CGLS against plain CGLS (a bounded training run)
        print("[bench] learned prior: pairs, training, PnP-CGLS vs CGLS ...", flush=True)
        from paper_2412_10129_amd import learned as LN
        learned = LN.quick_benchmark(log=lambda m: print(f"[bench] {m}", flush=True))
        print(f"[bench] learned: {learned['wall_s']} s", flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on one view ...", flush=True)
        cpu = cpu_baseline(geo, angles, x_h, y_h, kind)

    out = {
        "metric": "A/A^T voxel-view updates/s at 512^3 x 720",
        "value": float(f"{value:.4g}"),
        "unit": "voxel-view updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded U(0,1) volume and projections)",
        "config": {"workload": args.workload, "volume": list(geo.nVoxel), "views": nviews,
                   "detector": list(geo.nDetector), "projector": kind,
                   "step": "CGLS iteration: A, |q|^2, x/r update, A^T, |s|^2, p update"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "breakdown": breakdown,
        "learned": learned,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
