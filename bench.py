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

# MI355X datasheet figures: HBM3E bandwidth, and the non-packed FP32 vector
# issue rate derived from the unit counts (256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz = 39.32 T lane-instructions/s; the 157.3 TFLOP/s vector peak
# counts packed FMAs as 4 flops per lane-instruction, and this library is
# built without packed FP32)
PEAK_HBM_GBS = 8000.0
PEAK_VALU_TLI = 256 * 4 * 16 * 2.4e9 / 1e12

# algorithmic VALU lane-instructions per unit of work (minimum inner loops,
# non-packed):
#   Siddon A and A^T, per plane crossing: 2 compare/min to pick the next
#     plane, 1 sub for the length, 1 FMA to accumulate, 1 add to advance
#     alpha, 1 integer index step                                      = 6
#   interpolated A, per sample: 3 advance, 6 floor/fract, 7 lerps x 2,
#     1 accumulate                                                     = 24
#   interpolated A^T, per sample: 3 advance, 6 fract, 15 to form the 8
#     tent weights, 8 FMA scatters                                     = 32
#   FDK backprojection, per voxel-view update: 3 incremental numerators,
#     1 rcp, 2 mul, 2 weight, 4 floor/fract, 3 lerps x 2               = 18
INSTR = {"siddon_fwd": 6, "siddon_bwd": 6, "interp_fwd": 24, "interp_bwd": 32, "fdk_bp": 18}

# source file of each timed kernel (the HBM traffic recorded for a kernel in
# profiles/traffic.json is used only while that file is unchanged)
KERNEL_SOURCE = {"interp_fwd": "forward.hip", "siddon_fwd": "forward.hip", "interp_bwd": "backward.hip",
                 "siddon_bwd": "backward.hip", "fdk_bp": "fdk.hip", "fdk_filter": "fdk.hip"}


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


def _pmc_means(db_paths):
    """Per-kernel mean of every PMC counter over the dispatches in the given
    rocprofv3 databases (counters from several passes merged by kernel)."""
    import collections
    import re
    import sqlite3
    short = lambda n: re.sub(r"^void ", "", n.replace("ctmi::(anonymous namespace)::", "").split("(")[0]).strip()
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in db_paths:
        con = sqlite3.connect(path)
        rows = con.execute("select name, dispatch_id, counter_name, sum(counter_value) from pmc_events "
                           "group by name, dispatch_id, counter_name").fetchall()
        for name, _, cn, v in rows:
            acc[short(name)][cn].append(v)
    return {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in acc.items()}


def profile_derived(db_paths, cus=256, xcds=8):
    """Markdown table of derived per-kernel metrics from the counter passes
    (FETCH_SIZE; WRITE_SIZE, TCC_HIT_sum, TCC_MISS_sum; SQ counters with
    GRBM_GUI_ACTIVE): HBM bytes per dispatch scaled by the stream-copy
    kernel of the same run (it moves 2^30 bytes each way), L2 hit rate,
    VALU busy (rocprofv3's VALUBusy: SQ_ACTIVE_INST_VALU / CUs / cycles),
    VALU utilisation (active lanes per VALU instruction), VALU
    wave-instructions per CU-cycle, and LDS bank-conflict cycles per CU-cycle.
    GRBM_GUI_ACTIVE is summed over the XCDs; the per-XCD cycles divide it by
    their count."""
    m = _pmc_means(db_paths)
    cal = m.get("k_stream_copy", {})
    ff = (1 << 20) / cal["FETCH_SIZE"] if cal.get("FETCH_SIZE") else None
    wf = (1 << 20) / cal["WRITE_SIZE"] if cal.get("WRITE_SIZE") else None
    lines = [f"calibration: the 1 GiB stream copy reads FETCH_SIZE {cal.get('FETCH_SIZE', 0):.6g} KiB and "
             f"WRITE_SIZE {cal.get('WRITE_SIZE', 0):.6g} KiB (factors {ff and round(ff, 3)}, {wf and round(wf, 3)})", "",
             "| kernel | HBM read (GB) | HBM write (GB) | L2 hit % | VALU busy % | VALU util % | VALU instr / CU-cycle "
             "| LDS conflict cycles / CU-cycle |", "|---|---|---|---|---|---|---|---|"]
    for k in sorted(m):
        d = m[k]
        cyc = d.get("GRBM_GUI_ACTIVE", 0) / xcds
        f = lambda x: "" if x is None else f"{x:.3g}"
        rd = d["FETCH_SIZE"] * 1024 * ff / 1e9 if ff and "FETCH_SIZE" in d else None
        wr = d["WRITE_SIZE"] * 1024 * wf / 1e9 if wf and "WRITE_SIZE" in d else None
        hit = (100 * d["TCC_HIT_sum"] / (d["TCC_HIT_sum"] + d["TCC_MISS_sum"])
               if d.get("TCC_HIT_sum", 0) + d.get("TCC_MISS_sum", 0) > 0 else None)
        busy = 100 * d["SQ_ACTIVE_INST_VALU"] / cus / cyc if cyc and "SQ_ACTIVE_INST_VALU" in d else None
        util = (100 * d["SQ_THREAD_CYCLES_VALU"] / (64 * d["SQ_ACTIVE_INST_VALU"])
                if d.get("SQ_ACTIVE_INST_VALU") else None)
        ipc = d["SQ_INSTS_VALU"] / cus / cyc if cyc and "SQ_INSTS_VALU" in d else None
        ldsc = d["SQ_LDS_BANK_CONFLICT"] / cus / cyc if cyc and "SQ_LDS_BANK_CONFLICT" in d else None
        lines.append(f"| {k} | {f(rd)} | {f(wr)} | {f(hit)} | {f(busy)} | {f(util)} | {f(ipc)} | {f(ldsc)} |")
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


def _median_ms(torch, stream, fn, reps=10, warm=3):
    for _ in range(warm):
        fn()
    evs = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        evs.append((a, b))
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in evs]))


def measure_ceilings(torch, dev):
    """The two ceilings of the roofline, measured on this GPU: HBM bytes per
    second of a streaming copy of 2 GiB (read + write), and non-packed FP32
    lane-instructions per second of an FMA loop (16 independent chains per
    lane, 8192 workgroups of 256 lanes).  Medians of 10 launches."""
    import ctypes
    from paper_2412_10129_amd import _lib as L
    lib = L.lib()
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    n = 1 << 29
    a = torch.ones(n, dtype=torch.float32, device=dev)
    c = torch.empty_like(a)
    t_copy = _median_ms(torch, stream, lambda: L.check(lib.ctmi_ceiling_copy(
        ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(c.data_ptr()), n, sp)))
    if not bool(torch.equal(a, c)):
        raise RuntimeError("ceiling copy is wrong")
    del a, c
    blocks, iters = 8192, 4096
    out = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    t_fma = _median_ms(torch, stream, lambda: L.check(lib.ctmi_ceiling_fma(
        ctypes.c_void_p(out.data_ptr()), blocks, iters, sp)))
    lanes = blocks * 256 * int(lib.ctmi_ceiling_fma_per_lane(iters))
    return {"hbm_GBs": round(8.0 * n / (t_copy / 1e3) / 1e9, 1), "copy_ms": round(t_copy, 4),
            "valu_T_lane_instr_s": round(lanes / (t_fma / 1e3) / 1e12, 3), "fma_ms": round(t_fma, 4),
            "datasheet_hbm_GBs": PEAK_HBM_GBS, "datasheet_valu_T_lane_instr_s": round(PEAK_VALU_TLI, 3)}


def roof(t_ms, instr=0.0, nbytes=0.0, ceil=None):
    """Binding-roof fraction max(bytes / BW, instr / R) / t, with the measured
    ceilings and with the datasheet ones, and the bound it names."""
    t = t_ms / 1e3
    ent = {"ms": round(t_ms, 3)}
    if instr:
        ent["T_lane_instr_s"] = round(instr / t / 1e12, 3)
    if nbytes:
        ent["GB/s_alg"] = round(nbytes / t / 1e9, 1)
    for tag, bw, r in (("", ceil["hbm_GBs"] if ceil else None, ceil["valu_T_lane_instr_s"] if ceil else None),
                       ("_datasheet", PEAK_HBM_GBS, PEAK_VALU_TLI)):
        if bw is None:
            continue
        tb, ti = nbytes / (bw * 1e9), instr / (r * 1e12)
        ent["frac_roof" + tag] = round(max(tb, ti) / t, 4)
        if not tag:
            ent["bound"] = "alu" if ti >= tb else "hbm"
    return ent


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(geo, angles, x, y, kind):
    """The FP64 oracle on a sample of the workload: A and A^T on the first two
    views with every host thread, and on the first view with one thread
    (work is uniform over the views of a circular orbit, so the rate scales
    to the full 720 views)."""
    import oracle
    oracle._L()
    x64 = x.astype(np.float64)
    nt = oracle.num_threads()

    def timed(nviews):
        a = angles[:nviews]
        t0 = time.perf_counter()
        oracle.forward(geo, a, x64, kind)
        t1 = time.perf_counter()
        oracle.backward(geo, a, y[:nviews].astype(np.float64), kind)
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1
    fa, fb = timed(2)
    oracle.set_num_threads(1)
    try:
        sa, sb = timed(1)
    finally:
        oracle.set_num_threads(nt)
    upd = float(np.prod(geo.nVoxel))
    return {"value": 2 * 2 * upd / (fa + fb), "unit": "voxel-view updates/s", "cores": nt, "kind": "oracle",
            "sample": f"FP64 {kind} A and A^T on 2 of {len(angles)} views of the 512^3 workload with {nt} threads "
                      f"(A {fa:.1f} s, A^T {fb:.1f} s); rate scales to all views",
            "single_thread": {"value": 2 * upd / (sa + sb), "sample": f"1 view, 1 thread (A {sa:.1f} s, "
                                                                      f"A^T {sb:.1f} s)"},
            "cpu_model": _cpu_model(), "nproc": os.cpu_count()}


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
    ap.add_argument("--profile-derived", metavar="DB", nargs="+",
                    help="only print derived per-kernel metrics (HBM bytes, L2 hit rate, VALU busy and "
                         "utilisation, LDS conflicts) from rocprofv3 counter databases and exit")
    ap.add_argument("--profile-run", action="store_true",
                    help="run each rated kernel once on the workload (after a 1 GiB calibration copy) and exit: "
                         "the program profiled for kernel traces and counters")
    args = ap.parse_args()
    if args.profile_summary:
        print(profile_summary(args.profile_summary, top=args.top))
        return
    if args.profile_derived:
        print(profile_derived(args.profile_derived))
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
    if args.profile_run:
        import ctypes
        from paper_2412_10129_amd import algs as AL
        lib = ops.L.lib()
        cal = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        cal2 = torch.empty_like(cal)
        ops.L.check(lib.ctmi_ceiling_copy(ctypes.c_void_p(cal.data_ptr()), ctypes.c_void_p(cal2.data_ptr()), cal.numel(),
                                          ops._stream()))
        torch.cuda.synchronize()
        del cal, cal2
        gn = ops.dot(s, s)
        runs = [
            ("siddon_fwd", lambda: plan.forward(x, out=q, kind="siddon")),
            ("siddon_bwd", lambda: plan.backproject(b, out=s, kind="siddon")),
            ("interp_fwd", lambda: plan.forward(x, out=q, kind="interp")),
            ("interp_bwd", lambda: plan.backproject(b, out=s, kind="interp")),
            ("fdk_filter", lambda: plan.fdk_filter(b, out=q)),
            ("fdk_bp", lambda: plan.backproject(b, out=s, kind="fdk")),
            ("awtv_grad", lambda: ops.awtv_grad(x, out=p, delta=0.5)),
            ("tv_step", lambda: ops.tv_step(xs, p, gn, 1e-3)),
            ("cgls_xr", lambda: ops.cgls_xr(xs, p, r, q, slot(0, 0), slot(0, 1), slot(0, 2), ws)),
            ("cgls_p", lambda: ops.cgls_p(p, s, slot(0, 0), slot(1, 0))),
            ("dot_proj", lambda: dot_into(q, slot(1, 3))),
            ("em_ratio", lambda: ops.em_ratio(b, q, q)),
            ("em_update", lambda: ops.em_update(xs, p, s)),
        ]
        for name, fn in runs:
            fn()
            torch.cuda.synchronize()
            print(f"[bench] profile run: {name}", flush=True)
        print("[bench] profile run done", flush=True)
        return
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
    units = {"interp_fwd": samples, "interp_bwd": samples, "siddon_fwd": segments, "siddon_bwd": segments,
             "fdk_bp": upd}
    proj_bytes = 4.0 * (float(np.prod(geo.nVoxel)) + float(b.numel()))   # read one, write the other, once
    print("[bench] measuring the HBM and VALU ceilings ...", flush=True)
    ceil = measure_ceilings(torch, dev)
    print(f"[bench] ceilings: {ceil}", flush=True)
    kf, kb = f"{kind}_fwd", f"{kind}_bwd"
    dominant, t_dom = (kb, t_bwd) if t_bwd >= t_fwd else (kf, t_fwd)
    li = INSTR[dominant] * units[dominant]
    ach = li / (t_dom / 1e3) / 1e12
    rd = roof(t_dom, li, proj_bytes, ceil)
    roofline = {"bound": "alu", "kernel": dominant, "achieved": round(ach, 3), "peak": round(PEAK_VALU_TLI, 3),
                "unit": "T VALU lane-instr/s", "frac": round(ach / PEAK_VALU_TLI, 4),
                "traffic": recorded_traffic(dominant),
                "peak_measured": ceil["valu_T_lane_instr_s"], "frac_measured": rd["frac_roof"],
                "work_units": units[dominant], "lane_instr_per_unit": INSTR[dominant],
                "alg_bytes": proj_bytes, "avg_launch_ms": round(float(t_dom), 3), "ceilings": ceil}

    breakdown = {}
    if not args.no_breakdown:
        ops_list = [
            ("siddon_fwd", lambda: plan.forward(x, out=q, kind="siddon")),
            ("siddon_bwd", lambda: plan.backproject(b, out=s, kind="siddon")),
            ("interp_fwd", lambda: plan.forward(x, out=q, kind="interp")),
            ("interp_bwd", lambda: plan.backproject(b, out=s, kind="interp")),
            ("fdk_filter", lambda: plan.fdk_filter(b, out=q)),
            ("fdk_bp", lambda: plan.backproject(b, out=s, kind="fdk")),
        ]
        for name, fn in ops_list:
            t = _median_ms(torch, stream, fn, reps=3, warm=1)
            if name == "fdk_filter":
                ent = roof(t, 0.0, 8.0 * b.numel(), ceil)
            else:
                ent = roof(t, INSTR[name] * units[name], proj_bytes, ceil)
                ent["updates/s"] = float(f"{upd / (t / 1e3):.4g}")
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
            # CGLS vector steps of the timed iteration: x += a p, r -= a q with
            # |r|^2; p = s + b p; one FP64 norm of a projection-sized vector
            ("cgls_xr", lambda: ops.cgls_xr(xs, p, r, q, slot(0, 0), slot(0, 1), slot(0, 2), ws),
             12.0 * nvox + 12.0 * b.numel()),
            ("cgls_p", lambda: ops.cgls_p(bps, s, slot(0, 0), slot(1, 0)), 12.0 * nvox),
            ("dot_proj", lambda: dot_into(q, slot(1, 3)), 4.0 * b.numel()),
        ]
        for name, fn, nbytes in extra:
            t = _median_ms(torch, stream, fn, reps=3, warm=1)
            ent = roof(t, 0.0, nbytes, ceil)
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
        learned = LN.quick_benchmark(log=lambda m: print(f"[bench] {m}", flush=True), weights=LN.WEIGHTS)
        print(f"[bench] learned: {learned['wall_s']} s", flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on a sample of views ...", flush=True)
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
