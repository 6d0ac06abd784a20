"""The learned prior: a 3-D residual U-Net on libctmi's BF16 MFMA kernels.

The paper's section on data-driven methods notes that trained networks call
the projection operators; the network is this package's choice: 4 levels of
(16, 32, 64, 128) channels, two [3x3x3 conv + bias + ReLU] per level, 2x2x2
average pooling, stride-2 2x2x2 transposed convolutions, skip connections by
concatenation (upsampled channels first), and a 1x1x1 head added to the
input.  Weights and activations are BF16 with FP32 accumulation; the master
weights, their gradients and the Adam moments are FP32 in one flat device
buffer each.  Every arithmetic step is a libctmi kernel; torch only holds
device memory and the stream.

Activations are channels-last ``[N, D, H, W, C]`` BF16 tensors (torch
bfloat16, same bits as the library's uint16 BF16 values).
"""
from __future__ import annotations

import ctypes
import math
from typing import Dict, List, Optional, Tuple

import torch

import synth

from . import _lib as L
from .ops import _stream

CHANNELS = (16, 32, 64, 128)


def _p(t: Optional[torch.Tensor], offset_elems: int = 0):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr() + offset_elems * t.element_size())


def layers(channels=CHANNELS) -> List[Tuple[str, str, Tuple[int, int, int]]]:
    """(name, kind, weight shape) in forward order; kinds 'conv3'
    ([cout, 27, cin]), 'up2' ([cout, 8, cin]), 'head' ([1, 1, c])."""
    c = channels
    out, cin = [], 1
    for lvl, ch in enumerate(c):
        out += [(f"enc{lvl}a", "conv3", (ch, 27, cin)), (f"enc{lvl}b", "conv3", (ch, 27, ch))]
        cin = ch
    for lvl in range(len(c) - 2, -1, -1):
        out += [(f"up{lvl}", "up2", (c[lvl], 8, c[lvl + 1])), (f"dec{lvl}a", "conv3", (c[lvl], 27, 2 * c[lvl])),
                (f"dec{lvl}b", "conv3", (c[lvl], 27, c[lvl]))]
    out.append(("head", "head", (1, 1, c[0])))
    return out


class UNet:
    """Weights, Adam state and the forward / backward passes.

    ``forward(x)`` maps an FP32 volume batch ``[N, D, H, W]`` (D, H, W
    divisible by 8) to ``x + head(...)``.  ``train_step(x, target)`` runs
    forward, the MSE loss, backward and one Adam step, returning the loss.
    """

    def __init__(self, seed: int = 0, channels=CHANNELS, device=None, lr: float = 1e-3,
                 betas=(0.9, 0.999), eps: float = 1e-8):
        if channels[0] != 16:
            raise ValueError("the residual head reads 16 channels")
        self.ch = tuple(int(c) for c in channels)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.lr, self.betas, self.eps = float(lr), tuple(betas), float(eps)
        self.t = 0
        self.layers = layers(self.ch)
        # flat FP32 parameter buffer; the first convolution is stored padded
        # to 16 input channels (channels 1..15 stay zero: their inputs are 0)
        self._w: Dict[str, Tuple[int, Tuple[int, ...]]] = {}
        self._b: Dict[str, Tuple[int, int]] = {}
        off = 0
        for name, kind, shp in self.layers:
            st = (shp[0], shp[1], 16) if name == "enc0a" else shp
            n = st[0] * st[1] * st[2]
            self._w[name] = (off, st)
            off += (n + 3) // 4 * 4
            self._b[name] = (off, shp[0])
            off += (shp[0] + 3) // 4 * 4
        self.numel = off
        dev = self.device
        self.params = torch.zeros(off, dtype=torch.float32, device=dev)
        self.grads = torch.zeros(off, dtype=torch.float32, device=dev)
        self.m = torch.zeros(off, dtype=torch.float32, device=dev)
        self.v = torch.zeros(off, dtype=torch.float32, device=dev)
        specs = []
        for name, kind, shp in self.layers:
            fan = shp[1] * shp[2] if kind == "conv3" else shp[2]
            specs.append((shp, math.sqrt(2.0 / fan) if kind != "head" else 0.1 / math.sqrt(fan)))
        for (name, kind, shp), w0 in zip(self.layers, synth.normal_weights(seed, specs)):
            wv = self.w(name)
            wv[..., :shp[2]].copy_(torch.from_numpy(w0))
        # BF16 copies in the kernels' layouts
        self.wf: Dict[str, torch.Tensor] = {}
        self.wd: Dict[str, torch.Tensor] = {}
        for name, kind, _ in self.layers:
            st = self._w[name][1]
            self.wf[name] = torch.empty(st, dtype=torch.bfloat16, device=dev)
            if kind == "conv3" and name != "enc0a":
                self.wd[name] = torch.empty((st[2], 27, st[0]), dtype=torch.bfloat16, device=dev)
        self.pack()
        self._head_ws = torch.empty(L.lib().ctmi_unet_head_workspace_bytes() // 8 + 2, dtype=torch.float64, device=dev)
        self._sums = torch.zeros(18, dtype=torch.float64, device=dev)

    # -------------------------------------------------------------- params
    def w(self, name: str, grad: bool = False) -> torch.Tensor:
        off, st = self._w[name]
        buf = self.grads if grad else self.params
        return buf[off:off + st[0] * st[1] * st[2]].view(st)

    def b(self, name: str, grad: bool = False) -> torch.Tensor:
        off, n = self._b[name]
        buf = self.grads if grad else self.params
        return buf[off:off + n]

    def state_dict(self) -> Dict[str, torch.Tensor]:
        return {"params": self.params, "m": self.m, "v": self.v, "t": torch.tensor(self.t)}

    def load_state_dict(self, sd) -> None:
        self.params.copy_(sd["params"])
        self.m.copy_(sd["m"])
        self.v.copy_(sd["v"])
        self.t = int(sd["t"])
        self.pack()

    def pack(self, stream=None) -> None:
        """FP32 master weights -> the BF16 copies the kernels read."""
        lib, s = L.lib(), _stream(stream)
        for name, kind, _ in self.layers:
            st = self._w[name][1]
            if kind == "conv3":
                L.check(lib.ctmi_conv3d_pack_weights(_p(self.w(name)), st[0], st[2], _p(self.wf[name]),
                                                     _p(self.wd.get(name)), s))
            else:
                L.check(lib.ctmi_to_bf16(_p(self.w(name)), self.wf[name].numel(), _p(self.wf[name]), s))

    # ------------------------------------------------------------ helpers
    def _empty(self, n, d, h, w, c):
        return torch.empty((n, d, h, w, c), dtype=torch.bfloat16, device=self.device)

    def _conv(self, name, x0, x1=None, relu=True, stream=None):
        n, d, h, w, c0 = x0.shape
        c1 = 0 if x1 is None else x1.shape[-1]
        cout = self._w[name][1][0]
        out = self._empty(n, d, h, w, cout)
        L.check(L.lib().ctmi_conv3d_bf16_fwd(n, d, h, w, _p(x0), c0, c0, _p(x1), c1, c1 if c1 else 8,
                                             _p(self.wf[name]), _p(self.b(name)), cout, 1 if relu else 0, _p(out),
                                             cout, _stream(stream)))
        return out

    def _pool(self, x, stream=None):
        n, d, h, w, c = x.shape
        out = self._empty(n, d // 2, h // 2, w // 2, c)
        L.check(L.lib().ctmi_pool2(n, d // 2, h // 2, w // 2, c, _p(x), c, _p(out), c, _stream(stream)))
        return out

    def _up(self, name, x, stream=None):
        n, d, h, w, cin = x.shape
        cout = self._w[name][1][0]
        out = self._empty(n, 2 * d, 2 * h, 2 * w, cout)
        L.check(L.lib().ctmi_upsample2(n, d, h, w, _p(x), cin, cin, _p(self.wf[name]), _p(self.b(name)), cout,
                                       _p(out), cout, _stream(stream)))
        return out

    # ------------------------------------------------------------ forward
    def forward(self, x: torch.Tensor, keep: bool = False, stream=None):
        """D(x) for x [N, D, H, W] (or [D, H, W]) FP32 on the device."""
        squeeze = x.dim() == 3
        if squeeze:
            x = x[None]
        if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
            raise ValueError("x must be a contiguous float32 GPU tensor")
        n, d, h, w = x.shape
        if d % 8 or h % 8 or w % 8:
            raise ValueError("volume sizes must be multiples of 8 (three 2x poolings)")
        nl = len(self.ch)
        c = {}
        x0 = self._empty(n, d, h, w, 16)
        L.check(L.lib().ctmi_unet_pack_input(_p(x), x.numel(), _p(x0), _stream(stream)))
        c["x0"] = x0
        hcur, skips = x0, []
        for lvl in range(nl):
            a = self._conv(f"enc{lvl}a", hcur, stream=stream)
            hcur = self._conv(f"enc{lvl}b", a, stream=stream)
            c[f"enc{lvl}a"], c[f"enc{lvl}b"] = a, hcur
            if lvl < nl - 1:
                skips.append(hcur)
                hcur = self._pool(hcur, stream)
                c[f"pool{lvl + 1}"] = hcur
        for lvl in range(nl - 2, -1, -1):
            u = self._up(f"up{lvl}", hcur, stream)
            a = self._conv(f"dec{lvl}a", u, skips[lvl], stream=stream)
            hcur = self._conv(f"dec{lvl}b", a, stream=stream)
            c[f"up{lvl}"], c[f"dec{lvl}a"], c[f"dec{lvl}b"] = u, a, hcur
        out = torch.empty_like(x)
        L.check(L.lib().ctmi_unet_head(x.numel(), _p(x), _p(hcur), 16, 16, _p(self.wf["head"]), _p(self.b("head")),
                                       _p(out), _stream(stream)))
        c["x_in"] = x
        if squeeze:
            out = out[0]
        return (out, c) if keep else out

    __call__ = forward

    # ----------------------------------------------------------- backward
    def _ws(self, nbytes):
        return torch.empty((nbytes + 15) // 16 * 4 + 4, dtype=torch.float32, device=self.device)

    def _wgrad(self, name, x0, x1, dz, stream=None):
        n, d, h, w, c0 = x0.shape
        c1 = 0 if x1 is None else x1.shape[-1]
        cout = dz.shape[-1]
        lib = L.lib()
        nb = lib.ctmi_conv3d_wgrad_workspace_bytes(n, d, h, w, c0 + c1, cout)
        ws = self._ws(nb)
        L.check(lib.ctmi_conv3d_bf16_wgrad(n, d, h, w, _p(x0), c0, c0, _p(x1), c1, c1 if c1 else 8, _p(dz), cout,
                                           cout, _p(self.w(name, True)), _p(self.b(name, True)), 0, _p(ws),
                                           ws.numel() * 4, _stream(stream)))

    def _dgrad(self, name, dz, mask, stream=None):
        n, d, h, w, cout = dz.shape
        cin = self._w[name][1][2]
        dx = self._empty(n, d, h, w, cin)
        L.check(L.lib().ctmi_conv3d_bf16_dgrad(n, d, h, w, _p(dz), cout, cout, _p(self.wd[name]), cin, _p(mask),
                                               cin, _p(dx), cin, _stream(stream)))
        return dx

    def backward(self, cache, target: torch.Tensor, out: torch.Tensor, stream=None, record=None) -> torch.Tensor:
        """Gradients of mean((out - target)^2) into self.grads.  Returns a
        one-element device double holding sum((out - target)^2) (divide by
        the voxel count for the loss; nothing waits for the host).  With a
        dict `record`, the stored activation gradients are kept there:
        "dz.<layer>" at each layer's pre-activation (after its ReLU mask),
        "dcat<l>" at each concatenation, "dp<l>" at each pooled tensor."""
        rec = record if record is not None else {}
        lib, s = L.lib(), _stream(stream)
        nl = len(self.ch)
        x = cache["x_in"]
        n, d, h, w = x.shape
        target = target.reshape(x.shape)
        out = out.reshape(x.shape)
        top = cache["dec0b"]
        dz = self._empty(n, d, h, w, 16)
        hoff, _ = self._w["head"]
        L.check(lib.ctmi_unet_head_mse_bwd(x.numel(), _p(out), _p(target), _p(top), 16, _p(self.wf["head"]), _p(dz),
                                           16, _p(self._sums), _p(self.grads, hoff), _p(self._head_ws),
                                           self._head_ws.numel() * 8, s))
        # the head's bias gradient follows its 16 weights in the flat buffer
        assert self._b["head"][0] == hoff + 16
        skip_grads = {}
        for lvl in range(nl - 1):
            a = cache[f"dec{lvl}a"]
            rec[f"dz.dec{lvl}b"] = dz
            self._wgrad(f"dec{lvl}b", a, None, dz, stream)
            dz = self._dgrad(f"dec{lvl}b", dz, a, stream)
            rec[f"dz.dec{lvl}a"] = dz
            u, e = cache[f"up{lvl}"], cache[f"enc{lvl}b"]
            self._wgrad(f"dec{lvl}a", u, e, dz, stream)
            dcat = self._dgrad(f"dec{lvl}a", dz, None, stream)
            rec[f"dcat{lvl}"] = dcat
            cu = self.ch[lvl]
            skip_grads[lvl] = dcat
            below = cache[f"dec{lvl + 1}b"] if lvl + 1 < nl - 1 else cache[f"enc{nl - 1}b"]
            nb_, db_, hb_, wb_, cb = below.shape
            nbytes = lib.ctmi_upsample2_wgrad_workspace_bytes(nb_, db_, hb_, wb_, cb, cu)
            ws = self._ws(nbytes)
            L.check(lib.ctmi_upsample2_wgrad(nb_, db_, hb_, wb_, _p(below), cb, cb, _p(dcat), cu, 2 * cu,
                                             _p(self.w(f"up{lvl}", True)), _p(self.b(f"up{lvl}", True)), 0, _p(ws),
                                             ws.numel() * 4, s))
            dzb = self._empty(nb_, db_, hb_, wb_, cb)
            L.check(lib.ctmi_upsample2_dgrad(nb_, db_, hb_, wb_, _p(dcat), cu, 2 * cu, _p(self.wf[f"up{lvl}"]), cb,
                                             _p(below), cb, _p(dzb), cb, s))
            dz = dzb
        for lvl in range(nl - 1, -1, -1):
            a = cache[f"enc{lvl}a"]
            rec[f"dz.enc{lvl}b"] = dz
            self._wgrad(f"enc{lvl}b", a, None, dz, stream)
            dz = self._dgrad(f"enc{lvl}b", dz, a, stream)
            rec[f"dz.enc{lvl}a"] = dz
            inp = cache["x0"] if lvl == 0 else cache[f"pool{lvl}"]
            self._wgrad(f"enc{lvl}a", inp, None, dz, stream)
            if lvl == 0:
                break
            dp = self._dgrad(f"enc{lvl}a", dz, None, stream)
            rec[f"dp{lvl}"] = dp
            e = cache[f"enc{lvl - 1}b"]
            ne, de, he, we, ce = e.shape
            dze = self._empty(ne, de, he, we, ce)
            L.check(lib.ctmi_pool2_skip_grad(ne, de, he, we, ce, _p(e), ce, _p(dp), ce, _p(skip_grads[lvl - 1], ce),
                                             2 * ce, _p(dze), ce, s))
            dz = dze
        return self._sums[17:18]

    def adam_step(self, stream=None) -> None:
        self.t += 1
        L.check(L.lib().ctmi_adam_step(_p(self.params), _p(self.m), _p(self.v), _p(self.grads), self.numel,
                                       self.lr, self.betas[0], self.betas[1], self.eps, self.t, _stream(stream)))
        self.pack(stream)

    def train_step(self, x: torch.Tensor, target: torch.Tensor, stream=None) -> torch.Tensor:
        """One Adam step on mean((D(x) - target)^2); returns the device
        double sum of squared differences before the step."""
        out, cache = self.forward(x, keep=True, stream=stream)
        sq = self.backward(cache, target, out, stream)
        self.adam_step(stream)
        return sq
