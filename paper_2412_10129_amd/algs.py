"""Reconstruction drivers over libctmi kernels: FDK, CGLS and OS-SART.

The loops are host-side sequencing only; every arithmetic step is a libctmi
kernel, and the iteration scalars (norms, alpha, beta) stay on the device so
a loop never waits for the host.
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional

import numpy as np
import torch

from . import ops
from .ops import Plan


def fdk(plan: Plan, proj: torch.Tensor, wang: bool = False, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """FDK (section 2.1, direct methods): weight and ramp-filter each row,
    then the (DSO/U)^2-weighted voxel-driven backprojection."""
    q = plan.fdk_filter(proj, wang=wang)
    return plan.backproject(q, out=out, kind="fdk")


def _addr(t: torch.Tensor, i: int, j: int) -> int:
    return t.data_ptr() + 8 * (i * t.shape[1] + j)


def cgls(plan: Plan, b: torch.Tensor, niter: int, kind: str = "interp", x_gt: Optional[torch.Tensor] = None,
         x0: Optional[torch.Tensor] = None, sync: bool = True, snapshots=(), callback=None,
         state: Optional[dict] = None):
    """CGLS (Hestenes-Stiefel; the Krylov solvers of section 2.2.1).

    x0 = 0 (or the given start); r = b - A x0; s = A^T r; p = s; gamma = |s|^2;
    per iteration q = A p, delta = |q|^2, alpha = gamma/delta, x += alpha p,
    r -= alpha q, s = A^T r, gamma' = |s|^2, beta = gamma'/gamma, p = s + beta p.

    Returns (x, hist): hist holds per-iteration gamma, delta, |r|^2 and, given
    x_gt, the squared error and voxel count inside the FOV (the residual and
    error-norm histories of section 2.2.3).  With sync=False, hist holds the
    device tensors instead of host arrays.  hist["snapshots"][k] is a copy of
    the iterate after k iterations for every k in `snapshots`.  `callback(k,
    x)`, if given, runs on the host after iteration k (k = 1..niter) has been
    queued, with the iterate's device tensor (it may synchronize).

    hist["state"] is the resumable state after the last iteration: the
    iterate x, the residual r, the direction p, gamma = |A^T r|^2 (FP64, on
    the device) and the iteration count k.  Passing it back as `state`
    (possibly after save_state / load_state) continues the same iteration
    bit for bit: iteration numbers for `snapshots` and `callback` then count
    from state["k"].
    """
    dev = plan.device
    vol_shape, proj_shape = plan.vol_shape, plan.proj_shape()
    ws = ops._ws(dev)
    sc = torch.zeros((niter + 1, 3), dtype=torch.float64, device=dev)   # gamma_k, delta_k, |r_k|^2
    err = torch.zeros((niter, 2), dtype=torch.float64, device=dev)
    k0 = 0
    if state is not None:
        if x0 is not None:
            raise ValueError("cgls: give either x0 or state")
        x, r, p = (state[n].to(dev, torch.float32).clone() for n in ("x", "r", "p"))
        if x.shape != vol_shape or p.shape != vol_shape or r.shape != b.shape:
            raise ValueError("cgls: state shapes do not match the plan and b")
        sc[0, 0] = state["gamma"].to(dev, torch.float64).reshape(())
        k0 = int(state["k"])
        s = torch.empty_like(p)
    else:
        if x0 is None:
            x = torch.zeros(vol_shape, dtype=torch.float32, device=dev)
            r = b.clone()
        else:
            x = x0.clone()
            r = plan.forward(x, kind=kind)
            ops.axpby(1.0, b, -1.0, r)
        s = plan.backproject(r, kind=kind)
        p = s.clone()
        ops.L.check(ops.L.lib().ctmi_dot(ops._ptr(s, "s"), ops._ptr(s, "s"), s.numel(), _addr(sc, 0, 0),
                                         ws.data_ptr(), ws.numel() * 8, ops._stream()))
    q = torch.empty(proj_shape, dtype=torch.float32, device=dev)
    snaps = {int(k): None for k in snapshots}
    for k in range(niter):
        plan.forward(p, out=q, kind=kind)
        ops.L.check(ops.L.lib().ctmi_dot(ops._ptr(q, "q"), ops._ptr(q, "q"), q.numel(), _addr(sc, k, 1),
                                         ws.data_ptr(), ws.numel() * 8, ops._stream()))
        ops.cgls_xr(x, p, r, q, _addr(sc, k, 0), _addr(sc, k, 1), _addr(sc, k, 2), ws)
        plan.backproject(r, out=s, kind=kind)
        ops.L.check(ops.L.lib().ctmi_dot(ops._ptr(s, "s"), ops._ptr(s, "s"), s.numel(), _addr(sc, k + 1, 0),
                                         ws.data_ptr(), ws.numel() * 8, ops._stream()))
        ops.cgls_p(p, s, _addr(sc, k, 0), _addr(sc, k + 1, 0))
        if x_gt is not None:
            plan.fov_sq_err(x, x_gt, err[k])
        if k0 + k + 1 in snaps:
            snaps[k0 + k + 1] = x.clone()
        if callback is not None:
            callback(k0 + k + 1, x)
    st = {"x": x, "r": r, "p": p, "gamma": sc[niter, 0].clone(), "k": k0 + niter}
    hist = {"scalars": sc, "err": err, "snapshots": snaps, "state": st}
    if sync:
        h = sc.cpu().numpy()
        hist = {"gamma": h[:, 0], "delta": h[:niter, 1], "resid": np.sqrt(h[:niter, 2]),
                "alpha": h[:niter, 0] / np.where(h[:niter, 1] != 0, h[:niter, 1], np.inf),
                "beta": h[1:, 0] / np.where(h[:niter, 0] != 0, h[:niter, 0], np.inf), "snapshots": snaps,
                "state": st}
        stop = np.nonzero((h[:niter, 1] == 0) | (h[:niter, 0] == 0))[0]
        hist["stopped"] = int(stop[0]) if len(stop) else None
        if x_gt is not None:
            e = err.cpu().numpy()
            hist["sq_err"] = e[:, 0]
            hist["count"] = e[:, 1]
    return x, hist


def save_state(state: dict, f) -> None:
    """Write a solver state (tensors and integers, e.g. cgls's hist["state"]
    or an OS-SART checkpoint) with torch.save, tensors moved to the host."""
    torch.save({k: (v.detach().cpu() if isinstance(v, torch.Tensor) else v) for k, v in state.items()}, f)


def load_state(f, device=None) -> dict:
    """Read a state written by save_state (tensors only, no code: the safe
    loader), tensors on `device`."""
    sd = torch.load(f, map_location="cpu", weights_only=True)
    return {k: (v.to(device) if isinstance(v, torch.Tensor) and device is not None else v) for k, v in sd.items()}


def psnr_from_sq_err(sq_err, count, data_range: float):
    """PSNR = 10 log10(R^2 / MSE) over the FOV (section 2.2.3 error history)."""
    sq_err = np.asarray(sq_err, dtype=np.float64)
    mse = sq_err / np.asarray(count, dtype=np.float64)
    with np.errstate(divide="ignore"):
        return 10.0 * np.log10(data_range * data_range / mse)


def subsets(nviews: int, blocksize: int):
    """Consecutive blocks of views visited in order (section 2.2.2)."""
    return [(s, min(blocksize, nviews - s)) for s in range(0, nviews, blocksize)]


class OSSART:
    """OS-SART (section 2.2.2, Eq. 6 with the descent sign; SART row/column
    normalisation).  SART is blocksize 1, SIRT one block of all views.

    Precomputes W = 1/(A 1) for all views (one projection-sized array) and
    V_s = 1/(A_s^T 1) per block (one volume per block)."""

    def __init__(self, plan: Plan, blocksize: int, kind: str = "interp"):
        self.plan, self.kind = plan, kind
        self.blocks = subsets(plan.nviews, blocksize)
        dev = plan.device
        ones_v = torch.ones(plan.vol_shape, dtype=torch.float32, device=dev)
        self.W = plan.forward(ones_v, kind=kind)
        ops.recip_or_zero(self.W)
        self.V = []
        for v0, nb in self.blocks:
            ones_p = torch.ones(plan.proj_shape(nb), dtype=torch.float32, device=dev)
            V = plan.backproject(ones_p, kind=kind, view0=v0, nviews=nb)
            self.V.append(ops.recip_or_zero(V))
        mb = max(nb for _, nb in self.blocks)
        self._e = torch.empty(plan.proj_shape(mb), dtype=torch.float32, device=dev)
        self._bp = torch.empty(plan.vol_shape, dtype=torch.float32, device=dev)

    def sweep(self, x: torch.Tensor, b: torch.Tensor, lam: float = 1.0, nonneg: bool = True, first: int = 0,
              last: Optional[int] = None) -> torch.Tensor:
        """One pass over the blocks first..last-1 (all by default), in place
        on x.  A pass stopped after block j resumes from the iterate and
        first = j + 1 (checkpoint()) bit for bit."""
        plan = self.plan
        last = len(self.blocks) if last is None else last
        if not 0 <= first <= last <= len(self.blocks):
            raise ValueError("OSSART.sweep: block range out of bounds")
        for s in range(first, last):
            v0, nb = self.blocks[s]
            e = self._e[:nb]
            plan.forward(x, out=e, kind=self.kind, view0=v0, nviews=nb)
            ops.sart_residual(b[v0:v0 + nb], e, self.W[v0:v0 + nb], e)
            plan.backproject(e, out=self._bp, kind=self.kind, view0=v0, nviews=nb)
            ops.sart_update(x, self.V[s], self._bp, lam, nonneg)
        return x

    @staticmethod
    def checkpoint(x: torch.Tensor, passes: int, next_block: int) -> dict:
        """Resumable OS-SART state: the iterate, the completed passes and the
        next block of the current pass."""
        return {"x": x, "passes": int(passes), "next_block": int(next_block)}

    def run(self, b: torch.Tensor, niter: int, lam: float = 1.0, nonneg: bool = True,
            x0: Optional[torch.Tensor] = None) -> torch.Tensor:
        plan = self.plan
        x = torch.zeros(plan.vol_shape, dtype=torch.float32, device=plan.device) if x0 is None else x0.clone()
        for _ in range(niter):
            self.sweep(x, b, lam, nonneg)
        return x


def os_sart(plan: Plan, b: torch.Tensor, niter: int, blocksize: int, lam: float = 1.0, nonneg: bool = True,
            kind: str = "interp", x0: Optional[torch.Tensor] = None) -> torch.Tensor:
    return OSSART(plan, blocksize, kind).run(b, niter, lam, nonneg, x0)


class OSEM:
    """MLEM and OSEM (section 2.2, the update for the Kullback-Leibler data
    term; its ordered-subsets counterpart, section 2.2.2).  The update's
    normaliser is the sensitivity A_s^T 1 (a volume):
        x <- x * (1 / A_s^T 1) * A_s^T (b_s / A_s x)
    with the ratio 0 where A_s x <= 0 and x 0 where no ray of the block
    reaches the voxel.  MLEM is one block of all views.  Precomputes
    V_s = 1 / (A_s^T 1) per block (one volume per block)."""

    def __init__(self, plan: Plan, blocksize: Optional[int] = None, kind: str = "interp"):
        self.plan, self.kind = plan, kind
        self.blocks = subsets(plan.nviews, plan.nviews if blocksize is None else blocksize)
        dev = plan.device
        self.V = []
        for v0, nb in self.blocks:
            ones_p = torch.ones(plan.proj_shape(nb), dtype=torch.float32, device=dev)
            self.V.append(ops.recip_or_zero(plan.backproject(ones_p, kind=kind, view0=v0, nviews=nb)))
        mb = max(nb for _, nb in self.blocks)
        self._e = torch.empty(plan.proj_shape(mb), dtype=torch.float32, device=dev)
        self._bp = torch.empty(plan.vol_shape, dtype=torch.float32, device=dev)

    def step(self, x: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
        """One iteration (one pass over all blocks), in place on x."""
        plan = self.plan
        for s, (v0, nb) in enumerate(self.blocks):
            e = self._e[:nb]
            plan.forward(x, out=e, kind=self.kind, view0=v0, nviews=nb)
            ops.em_ratio(b[v0:v0 + nb], e, e)
            plan.backproject(e, out=self._bp, kind=self.kind, view0=v0, nviews=nb)
            ops.em_update(x, self.V[s], self._bp)
        return x

    def run(self, b: torch.Tensor, niter: int, x0: Optional[torch.Tensor] = None) -> torch.Tensor:
        plan = self.plan
        x = torch.ones(plan.vol_shape, dtype=torch.float32, device=plan.device) if x0 is None else x0.clone()
        for _ in range(niter):
            self.step(x, b)
        return x


def mlem(plan: Plan, b: torch.Tensor, niter: int, kind: str = "interp",
         x0: Optional[torch.Tensor] = None) -> torch.Tensor:
    return OSEM(plan, None, kind).run(b, niter, x0)


def osem(plan: Plan, b: torch.Tensor, niter: int, blocksize: int, kind: str = "interp",
         x0: Optional[torch.Tensor] = None) -> torch.Tensor:
    return OSEM(plan, blocksize, kind).run(b, niter, x0)


class ASDPOCS:
    """ASD-POCS and OS-ASD-POCS (section 2.2: the POCS class, a data step
    alternated with adaptive TV steepest descent; OS version over blocks of
    views, section 2.2.2; adaptive-weighted TV for finite delta, section
    2.2.3), following Sidky and Pan.  Per iteration: one OS-SART pass with
    step lam (x >= 0 after each block if nonneg); dd = |A x - b| and
    dp = |change of the pass| (the first iteration sets the TV step
    dtvg = alpha dp); ng steps x -= dtvg g / |g|, g the (Aw)TV gradient;
    dg = |change of the TV steps|; if dg > rmax dp and dd > eps_data,
    dtvg *= alpha_red; lam *= lam_red.  The three norms are read on the host
    once per iteration (the step rule needs them); everything else stays on
    the device."""

    def __init__(self, plan: Plan, blocksize: int = 1, kind: str = "interp"):
        self.plan, self.kind = plan, kind
        self.sart = OSSART(plan, blocksize, kind)
        dev = plan.device
        self._prev = torch.empty(plan.vol_shape, dtype=torch.float32, device=dev)
        self._g = torch.empty(plan.vol_shape, dtype=torch.float32, device=dev)
        self._res = torch.empty(plan.proj_shape(), dtype=torch.float32, device=dev)
        self._gn = torch.empty(1, dtype=torch.float64, device=dev)
        self._nrm = torch.empty(3, dtype=torch.float64, device=dev)
        self._ws = ops._ws(dev)

    def _dist2(self, x: torch.Tensor, ref: torch.Tensor, slot: int) -> None:
        """|x - ref|^2 into self._nrm[slot]; ref is overwritten by x - ref."""
        ops.axpby(1.0, x, -1.0, ref)
        ops.dot(ref, ref, out=self._nrm[slot:slot + 1], ws=self._ws)

    def run(self, b: torch.Tensor, niter: int, lam: float = 1.0, lam_red: float = 0.99, alpha: float = 0.002,
            alpha_red: float = 0.95, ng: int = 20, rmax: float = 0.95, eps_data: float = 0.0,
            delta: float = float("inf"), eps_tv: float = 1e-8, nonneg: bool = True,
            x0: Optional[torch.Tensor] = None) -> torch.Tensor:
        plan = self.plan
        x = torch.zeros(plan.vol_shape, dtype=torch.float32, device=plan.device) if x0 is None else x0.clone()
        dtvg = None
        for _ in range(niter):
            self._prev.copy_(x)
            self.sart.sweep(x, b, lam, nonneg)
            plan.forward(x, out=self._res, kind=self.kind)
            self._dist2(b, self._res, 0)            # |b - A x|^2 (sign irrelevant)
            self._dist2(x, self._prev, 1)           # |x - x_prev|^2
            self._prev.copy_(x)
            for _ in range(ng):
                ops.awtv_grad(x, out=self._g, delta=delta, eps=eps_tv)
                ops.dot(self._g, self._g, out=self._gn, ws=self._ws)
                if dtvg is None:
                    # the first TV step length needs dp (one host read)
                    dtvg = alpha * float(self._nrm[1].item()) ** 0.5
                ops.tv_step(x, self._g, self._gn, dtvg)
            self._dist2(x, self._prev, 2)           # |x - x_before_tv|^2
            dd, dp, dg = (float(v) ** 0.5 for v in self._nrm.cpu())
            if dtvg is None:
                dtvg = alpha * dp
            if dg > rmax * dp and dd > eps_data:
                dtvg *= alpha_red
            lam *= lam_red
        return x


def asd_pocs(plan: Plan, b: torch.Tensor, niter: int, blocksize: int = 1, kind: str = "interp",
             **kw) -> torch.Tensor:
    """ASD-POCS (blocksize 1: SART data steps); OS-ASD-POCS for blocksize > 1;
    AwTV-ASD-POCS with a finite delta."""
    return ASDPOCS(plan, blocksize, kind).run(b, niter, **kw)


def pnp_cgls(plan: Plan, b: torch.Tensor, niter: int, denoiser, every: int = 5, ratio: float = 1.05,
             kind: str = "interp", x_gt: Optional[torch.Tensor] = None, data_range: Optional[float] = None,
             timing: bool = False, keep: Optional[list] = None):
    """CGLS with a plug-and-play denoiser step (the learned prior inside the
    Krylov solver of section 2.2.1).

    CGLS from x = 0; after every `every` iterations, x' = denoiser(x) and
    r' = b - A x'; when |r'| <= ratio |r| (r the CGLS residual vector) CGLS
    restarts at x' (r = r', s = p = A^T r', gamma = |s|^2), otherwise the
    proposal is dropped and CGLS continues unchanged.  One host
    synchronisation per proposal takes the decision.

    Returns (x, hist): per-iteration residual norms, the proposals' ratios and
    decisions, with x_gt the FOV squared errors (and PSNR given data_range),
    and with timing=True the per-iteration solver time in ms (GPU events
    around each iteration's kernels, error bookkeeping excluded).  When
    `keep` is a list, a device copy of every iterate is appended to it
    (outside the timed region), for judging them afterwards.
    """
    dev = plan.device
    ws = ops._ws(dev)
    npro = niter // every
    g = torch.zeros(niter + npro + 2, dtype=torch.float64, device=dev)     # gamma slots
    sc = torch.zeros((niter, 3), dtype=torch.float64, device=dev)          # delta_k, |r_k|^2, |r'|^2
    err = torch.zeros((niter, 2), dtype=torch.float64, device=dev)
    x = torch.zeros(plan.vol_shape, dtype=torch.float32, device=dev)
    r = b.clone()
    s = plan.backproject(r, kind=kind)
    p = s.clone()
    q = torch.empty(plan.proj_shape(), dtype=torch.float32, device=dev)
    rd = torch.empty_like(q)
    lib, st = ops.L.lib(), ops._stream()

    def dot_into(a, addr):
        ops.L.check(lib.ctmi_dot(ops._ptr(a, "a"), ops._ptr(a, "a"), a.numel(), ctypes.c_void_p(addr),
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel() * 8, st))

    gaddr = lambda i: g.data_ptr() + 8 * i
    dot_into(s, gaddr(0))
    gi = 0
    ratios, accepted, resid_from_proposal = [], [], {}
    ev = []
    for k in range(niter):
        if timing:
            e0 = torch.cuda.Event(enable_timing=True)
            e0.record()
        plan.forward(p, out=q, kind=kind)
        dot_into(q, _addr(sc, k, 0))
        ops.cgls_xr(x, p, r, q, gaddr(gi), _addr(sc, k, 0), _addr(sc, k, 1), ws)
        plan.backproject(r, out=s, kind=kind)
        dot_into(s, gaddr(gi + 1))
        ops.cgls_p(p, s, gaddr(gi), gaddr(gi + 1))
        gi += 1
        if (k + 1) % every == 0:
            xd = denoiser(x)
            plan.forward(xd, out=rd, kind=kind)
            ops.axpby(1.0, b, -1.0, rd)
            dot_into(rd, _addr(sc, k, 2))
            h = sc[k].cpu().numpy()
            qk = math.sqrt(h[2] / h[1]) if h[1] > 0 else math.inf
            ratios.append(qk)
            accepted.append(bool(qk <= ratio))
            if accepted[-1]:
                x.copy_(xd)
                r.copy_(rd)
                plan.backproject(r, out=s, kind=kind)
                p.copy_(s)
                dot_into(s, gaddr(gi + 1))
                gi += 1
                resid_from_proposal[k] = math.sqrt(h[2])
        if timing:
            e1 = torch.cuda.Event(enable_timing=True)
            e1.record()
            ev.append((e0, e1))
        if x_gt is not None:
            plan.fov_sq_err(x, x_gt, err[k])
        if keep is not None:
            keep.append(x.clone())
    h = sc.cpu().numpy()
    resid = np.sqrt(h[:, 1])
    for k, v in resid_from_proposal.items():
        resid[k] = v
    hist = {"resid": resid, "ratios": ratios, "accepted": accepted}
    if x_gt is not None:
        e = err.cpu().numpy()
        hist["sq_err"], hist["count"] = e[:, 0], e[:, 1]
        if data_range is not None:
            hist["psnr"] = psnr_from_sq_err(e[:, 0], e[:, 1], data_range)
    if timing:
        torch.cuda.synchronize()
        hist["ms"] = np.array([a.elapsed_time(bb) for a, bb in ev])
    return x, hist
