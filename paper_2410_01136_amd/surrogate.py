"""Coordinate-MLP surrogate of the march's fields (training and export).

The network maps a position to (B_x, B_y, B_z [uG], ln n_e, ln N0):
x^ = 2 (r - lo) / (hi - lo) - 1, 16 Gaussian Fourier frequency vectors b_f
(N(0, 4^2) per component, seeded) giving sin(2 pi b_f.x^) and cos(2 pi b_f.x^)
(32 features), 4 hidden layers of width 128 with a cubic-gated linear unit
(the shape of GELU at a fraction of its cost on the vector units, see
act_cubic), and a linear output.  It is trained in PyTorch on points sampled uniformly in the box whose
targets are the gridded fields evaluated by the library itself (trilinear
interpolation on the GPU), with a mean-squared loss on standardised outputs.

For inference the weights are rounded to FP16 and packed by syn_mlp_pack for
the fused MFMA march kernel (FP32 biases and sums), which evaluates the gate in
FP16.  The plain evaluator (the field the surrogate
stands in for) judges its map error and is the fallback: `judge` marches a
probe geometry with both and keeps the surrogate only within stated error
bounds.  `reference_eval` repeats that FP16 computation in plain PyTorch
(FP16-rounded weights and layer inputs, FP32 sums and biases, the gate in FP16)
as the check of the kernel.
"""
from __future__ import annotations

import ctypes
import math
import time
from dataclasses import dataclass
from typing import Callable, Optional

import numpy as np
import torch
import torch.nn as nn

from . import binding as sm

def act_cubic(x: torch.Tensor) -> torch.Tensor:
    """Cubic-gated linear unit: x S(s) with s = clamp(x / 4 + 1/2, 0, 1) and
    S(s) = s^2 (3 - 2 s), a smooth gate from 0 (x <= -2) to 1 (x >= 2) shaped
    like the normal CDF of GELU (value 1/2 and slope 3/8 at 0).  The network is
    trained and evaluated with it."""
    s = torch.clamp(x * 0.25 + 0.5, 0.0, 1.0)
    return x * (s * s * (3.0 - 2.0 * s))


def layer_f16(acc: torch.Tensor, bias: torch.Tensor) -> torch.Tensor:
    """The kernel's bias and activation: the FP32 bias added to the FP32
    accumulator, the sum rounded to FP16 and the gate applied in FP16
    arithmetic (every operation rounded to FP16); returned as FP32 values."""
    x = (acc + bias.float()).to(torch.float16)
    s = torch.clamp(x * 0.25 + 0.5, 0.0, 1.0)
    return (x * (s * s * (3.0 - 2.0 * s))).to(torch.float32)


class CubicGate(nn.Module):
    def forward(self, x: torch.Tensor) -> torch.Tensor:
        return act_cubic(x)


N_FOURIER = 16
WIDTH = 128
N_HIDDEN = 4
N_OUT = 5


class FieldMLP(nn.Module):
    def __init__(self, lo, hi, seed: int = 4002, freq_sigma: float = 4.0):
        super().__init__()
        g = torch.Generator().manual_seed(seed)
        self.register_buffer("lo", torch.tensor(lo, dtype=torch.float32))
        self.register_buffer("hi", torch.tensor(hi, dtype=torch.float32))
        self.register_buffer("fourier", torch.randn(N_FOURIER, 3, generator=g) * freq_sigma)
        layers = [nn.Linear(2 * N_FOURIER, WIDTH)] + [nn.Linear(WIDTH, WIDTH) for _ in range(N_HIDDEN - 1)]
        self.hidden = nn.ModuleList(layers)
        self.out = nn.Linear(WIDTH, N_OUT)
        with torch.random.fork_rng(devices=[]):
            torch.manual_seed(seed + 1)
            for m in list(self.hidden) + [self.out]:
                nn.init.kaiming_uniform_(m.weight, a=math.sqrt(5))
                bound = 1.0 / math.sqrt(m.weight.shape[1])
                nn.init.uniform_(m.bias, -bound, bound)
        self.act = CubicGate()
        # output de-standardisation (set from the training targets)
        self.register_buffer("out_scale", torch.ones(N_OUT))
        self.register_buffer("out_shift", torch.zeros(N_OUT))

    def features(self, r: torch.Tensor) -> torch.Tensor:
        x = 2.0 * (r - self.lo) / (self.hi - self.lo) - 1.0
        t = 2.0 * math.pi * (x @ self.fourier.T)
        return torch.cat([torch.sin(t), torch.cos(t)], dim=-1)

    def forward_std(self, r: torch.Tensor) -> torch.Tensor:
        h = self.features(r)
        for lin in self.hidden:
            h = self.act(lin(h))
        return self.out(h)

    def forward(self, r: torch.Tensor) -> torch.Tensor:
        """(B_x, B_y, B_z, ln n_e, ln N0)."""
        return self.forward_std(r) * self.out_scale + self.out_shift

    def export(self):
        """FP32 numpy arrays in the layout syn_mlp_pack expects (output layer with
        the de-standardisation folded in)."""
        f = lambda t: np.ascontiguousarray(t.detach().float().cpu().numpy())
        w_h = np.stack([f(l.weight) for l in self.hidden[1:]])
        b_h = np.stack([f(l.bias) for l in self.hidden[1:]])
        w_out = f(self.out.weight) * f(self.out_scale)[:, None]
        b_out = f(self.out.bias) * f(self.out_scale) + f(self.out_shift)
        return dict(fourier=f(self.fourier), w_in=f(self.hidden[0].weight), b_in=f(self.hidden[0].bias),
                    w_h=w_h, b_h=b_h, w_out=np.ascontiguousarray(w_out, dtype=np.float32),
                    b_out=np.ascontiguousarray(b_out, dtype=np.float32))


def pack(model: FieldMLP, device="cuda") -> torch.Tensor:
    """FP16-packed weights on the device (layout of syn_mlp_pack)."""
    e = model.export()
    nbytes = int(sm.syn_mlp_packed_bytes())
    host = np.zeros(nbytes, dtype=np.uint8)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    sm.check(sm.syn_mlp_pack(ptr(e["fourier"]), ptr(e["w_in"]), ptr(e["b_in"]), ptr(e["w_h"]),
                             ptr(e["b_h"]), ptr(e["w_out"]), ptr(e["b_out"]), host.ctypes.data),
             "syn_mlp_pack")
    return torch.from_numpy(host).to(device)


def mlp_field(model: FieldMLP, packed: torch.Tensor, alpha: float = 3.0) -> sm.Field:
    th = np.zeros(16)
    th[12] = alpha
    return sm.Field(sm.FIELD_MLP, th, lo=model.lo.tolist(), hi=model.hi.tolist(), mlp=packed)


def _f16(t: torch.Tensor) -> torch.Tensor:
    return t.to(torch.float16).to(torch.float32)


@torch.no_grad()
def reference_eval(model: FieldMLP, r: torch.Tensor) -> torch.Tensor:
    """The kernel's arithmetic in plain PyTorch: FP16-rounded weights and layer
    inputs, FP32 sums and biases, cubic gate in FP16; returns (B_x, B_y, B_z, n_e, N0)."""
    e = model.export()
    dev = r.device
    T = lambda a: torch.from_numpy(a).to(dev)
    x = 2.0 * (r.float() - model.lo.to(dev)) / (model.hi.to(dev) - model.lo.to(dev)) - 1.0
    t = x @ T(e["fourier"]).T
    h = torch.cat([torch.sin(2 * math.pi * t), torch.cos(2 * math.pi * t)], dim=-1)
    ws = [T(e["w_in"])] + [T(w) for w in e["w_h"]]
    bs = [T(e["b_in"])] + [T(b) for b in e["b_h"]]
    h = _f16(h)
    for w, b in zip(ws, bs):
        h = layer_f16(h @ _f16(w).T, b)
    o = h @ _f16(T(e["w_out"])).T + T(e["b_out"])
    return torch.cat([o[:, :3], torch.exp(o[:, 3:5])], dim=-1)


@dataclass
class TrainResult:
    model: FieldMLP
    seconds: float
    final_loss: float
    steps: int


def train(target_fn: Callable[[torch.Tensor], torch.Tensor], lo, hi, n_points: int = 10_000_000,
          steps: int = 3000, batch: int = 65536, lr: float = 2e-3, seed: int = 4001,
          init_seed: int = 4002, device="cuda", log: Optional[Callable[[str], None]] = None) -> TrainResult:
    """Fits the surrogate to target_fn(r) -> (B_x, B_y, B_z, n_e, N0) on n_points
    uniform points of the box (seeded)."""
    t0 = time.time()
    g = torch.Generator(device="cpu").manual_seed(seed)
    lo_t = torch.tensor(lo, dtype=torch.float32)
    hi_t = torch.tensor(hi, dtype=torch.float32)
    pts = (lo_t + (hi_t - lo_t) * torch.rand(n_points, 3, generator=g)).to(device)
    tgt = []
    for i in range(0, n_points, 1 << 20):
        f = target_fn(pts[i:i + (1 << 20)].contiguous())
        tgt.append(torch.cat([f[:, :3], torch.log(torch.clamp(f[:, 3:5], min=1e-30))], dim=-1))
    tgt = torch.cat(tgt)
    model = FieldMLP(lo, hi, seed=init_seed).to(device)
    shift = tgt.mean(0)
    scale = tgt.std(0)
    shift[:3] = 0.0
    scale[:3] = tgt[:, :3].std()  # one scale for the vector components
    model.out_scale.copy_(scale)
    model.out_shift.copy_(shift)
    ystd = (tgt - shift) / scale
    opt = torch.optim.Adam(model.parameters(), lr=lr)
    sched = torch.optim.lr_scheduler.OneCycleLR(opt, max_lr=lr, total_steps=steps, pct_start=0.1)
    gi = torch.Generator(device=device).manual_seed(seed + 7)
    loss_v = float("nan")
    for it in range(steps):
        idx = torch.randint(0, n_points, (batch,), device=device, generator=gi)
        loss = ((model.forward_std(pts[idx]) - ystd[idx]) ** 2).mean()
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        sched.step()
        if it % 500 == 0 or it == steps - 1:
            loss_v = loss.item()
            if log:
                log(f"surrogate step {it}: loss {loss_v:.4e}")
    return TrainResult(model=model, seconds=time.time() - t0, final_loss=loss_v, steps=steps)


@dataclass
class Judged:
    """The field to march with after the plain evaluator judged the surrogate:
    the surrogate's own field if its map error on the probe stayed within the
    bounds, else the plain field it stands in for (the fallback)."""
    field: sm.Field
    used_surrogate: bool
    error: dict


def map_error(maps: torch.Tensor, ref: torch.Tensor) -> dict:
    """Relative rms errors of I, Q, U and PI of maps [n_freq][3][npix] against ref."""
    a, b = maps.double(), ref.double()
    rms = lambda x: float(torch.sqrt((x * x).mean()))
    pa, pb = torch.hypot(a[:, 1], a[:, 2]), torch.hypot(b[:, 1], b[:, 2])
    return {"I_rel_rms": rms(a[:, 0] - b[:, 0]) / rms(b[:, 0]),
            "Q_rel_rms": rms(a[:, 1] - b[:, 1]) / rms(b[:, 1]),
            "U_rel_rms": rms(a[:, 2] - b[:, 2]) / rms(b[:, 2]),
            "PI_rel_rms": rms(pa - pb) / rms(pb)}


def judge(surrogate: sm.Field, plain: sm.Field, probe: sm.SynGeom, max_I_rel_rms: float = 0.05,
          max_PI_rel_rms: float = 0.10) -> Judged:
    """Marches the probe geometry (e.g. the target sky at a lower N_side) with
    both fields; the plain evaluator's maps are the reference.  Returns the
    surrogate's field if its relative rms errors of I and PI are within the
    bounds, otherwise the plain field."""
    m = sm.forward(probe, surrogate)
    r = sm.forward(probe, plain)
    err = map_error(m, r)
    ok = err["I_rel_rms"] <= max_I_rel_rms and err["PI_rel_rms"] <= max_PI_rel_rms
    err["bounds"] = {"I_rel_rms": max_I_rel_rms, "PI_rel_rms": max_PI_rel_rms}
    return Judged(field=surrogate if ok else plain, used_surrogate=ok, error=err)
