"""Training driver of the learned hyper-diffusion coefficient.

The network (four periodic 3x3 convolutions, BF16 weights, FP32
accumulation; see include/sacx.h) runs entirely in the HIP library: this
module only owns the torch buffers, draws the training schedule and calls
the library's forward, backward and Adam kernels.  Training data are
solver-generated: seeded Orszag-Tang runs whose states are turned into
network inputs (sacx_cnn_inputs) and plain coefficient-ratio targets
(sacx_hd_ratio_fields) on the device.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import sacx as sx

LAYERS = ((6, 32), (32, 32), (32, 32), (32, 10))
IDENTITY_NORM = (0.0,) * 6 + (1.0,) * 6


def init_theta(seed: int = 0, device="cuda") -> torch.Tensor:
    """He-initialised FP32 parameter vector (w0 b0 ... w3 b3), seeded; the
    output bias starts at -4 so the initial prediction is small (R is mostly
    near 0 on resolved flows)."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    parts = []
    for l, (ci, co) in enumerate(LAYERS):
        std = math.sqrt(2.0 / (9 * ci))
        parts.append(torch.randn(co * ci * 9, generator=g, dtype=torch.float64) * std)
        b = torch.zeros(co, dtype=torch.float64)
        if l == len(LAYERS) - 1:
            b -= 4.0
        parts.append(b)
    th = torch.cat(parts).to(torch.float32)
    assert th.numel() == sx.CNN_NPARAM
    return th.to(device)


class Network:
    """Parameters, packed weights and Adam state of one network on one device."""

    def __init__(self, theta: Optional[torch.Tensor] = None, seed: int = 0, device="cuda"):
        dev = torch.device(device)
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.theta = (init_theta(seed, dev) if theta is None else theta.to(dev, torch.float32)).contiguous()
        self.packed = torch.empty(sx.CNN_PACKED_BYTES, dtype=torch.uint8, device=dev)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.grad = torch.zeros_like(self.theta)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.step = 0
        self._bufs: Dict[Tuple[int, int, int], Dict[str, torch.Tensor]] = {}
        self.pack()

    def pack(self):
        sx.cnn_pack(self.theta, self.packed)

    def _buffers(self, n: int, h: int, w: int) -> Dict[str, torch.Tensor]:
        key = (n, h, w)
        if key not in self._bufs:
            sz = sx.cnn_buffer_sizes(n, h, w)
            self._bufs[key] = {
                "act": torch.empty(sz["act"], dtype=torch.uint8, device=self.device),
                "out": torch.empty((n, 10, h, w), dtype=torch.float32, device=self.device),
                "work": torch.empty(sz["work"], dtype=torch.uint8, device=self.device),
            }
        return self._bufs[key]

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        """x: (n, h, w, 8) bf16 -> predicted ratio planes (n, 10, h, w)."""
        n, h, w = x.shape[:3]
        b = self._buffers(n, h, w)
        sx.cnn_forward(self.packed, x, b["act"], b["out"])
        return b["out"]

    def loss_of(self, x: torch.Tensor, target: torch.Tensor, weight: Optional[torch.Tensor] = None) -> float:
        """(Weighted) mean squared error of the prediction on a batch (synchronises)."""
        n, h, w = x.shape[:3]
        b = self._buffers(n, h, w)
        sx.cnn_forward(self.packed, x, b["act"], b["out"])
        sx.cnn_backward(self.packed, x, b["act"], b["out"], target, b["work"], self.grad, self.loss, weight)
        return float(self.loss.item())

    def train_step(self, x: torch.Tensor, target: torch.Tensor, lr: float,
                   weight: Optional[torch.Tensor] = None) -> torch.Tensor:
        """One forward/backward/Adam step on a batch; returns the (pre-step)
        loss as a device tensor (no synchronisation)."""
        n, h, w = x.shape[:3]
        b = self._buffers(n, h, w)
        sx.cnn_forward(self.packed, x, b["act"], b["out"])
        sx.cnn_backward(self.packed, x, b["act"], b["out"], target, b["work"], self.grad, self.loss, weight)
        self.step += 1
        sx.cnn_adam(self.theta, self.m, self.v, self.grad, self.step, lr)
        self.pack()
        return self.loss


@dataclasses.dataclass
class Dataset:
    """Network inputs, plain-ratio targets and flux weights grouped by image
    size.  The weight of a face is (|d1| / D)^2, d1 its first difference and
    D the largest |d1| of the plane in that snapshot: the squared error of the
    flux-weighted check metric is the weighted squared ratio error."""
    norm: Tuple[float, ...]
    x: Dict[int, torch.Tensor]   # side -> (m, side, side, 8) bf16
    y: Dict[int, torch.Tensor]   # side -> (m, 10, side, side) float32
    w: Dict[int, torch.Tensor]   # side -> (m, 10, side, side) float32
    meta: Dict


def flux_weights(d1: torch.Tensor) -> torch.Tensor:
    """(|d1| / max |d1| of each plane)^2 (0 on a plane without differences)."""
    a = d1.abs()
    D = a.amax(dim=(-2, -1), keepdim=True)
    return torch.where(D > 0, a / torch.where(D > 0, D, torch.ones_like(D)), torch.zeros_like(a)) ** 2


def input_norm(states: Sequence["sx.Solver"]) -> Tuple[float, ...]:
    """Shift (mean) and scale (1 / std) of the six raw inputs over some states."""
    acc = []
    for s in states:
        x = s.cnn_inputs(IDENTITY_NORM).to(torch.float32)[..., :6].reshape(-1, 6)
        acc.append(x)
    x = torch.cat(acc)
    mu = x.mean(dim=0)
    sd = x.std(dim=0).clamp_min(1e-6)
    return tuple(float(v) for v in mu) + tuple(float(1.0 / v) for v in sd)


def ot_solver(side: int, b0: float, precision=sx.FP64, device="cuda") -> "sx.Solver":
    import workloads as W
    return sx.Solver.from_problem(W.orszag_tang(side, b0_scale=b0), precision=precision, device=device)


def generate(sides: Sequence[int] = (256, 384, 512), seeds: Sequence[int] = tuple(range(1, 9)),
             snap_every=10, t_end: float = 3.0, max_snaps: int = 0, precision=sx.FP64,
             norm: Optional[Sequence[float]] = None, device="cuda", log=None) -> Dataset:
    """Seeded Orszag-Tang runs (B0 scaled by U(0.5, 1.5) from each seed),
    snapshots every `snap_every` steps until t_end (an int, or a dict from
    side to interval: a 1024^2 snapshot takes about 100 MB)."""
    b0s = {s: float(np.random.default_rng(s).uniform(0.5, 1.5)) for s in seeds}
    if norm is None:
        probe = [ot_solver(min(sides), b0s[s], precision, device) for s in seeds[:2]]
        for p in probe:
            p.advance(200, t_end=t_end)
        norm = input_norm(probe)
        for p in probe:
            p.close()
    xs: Dict[int, List[torch.Tensor]] = {}
    ys: Dict[int, List[torch.Tensor]] = {}
    ws: Dict[int, List[torch.Tensor]] = {}
    for side in sides:
        every = snap_every[side] if isinstance(snap_every, dict) else snap_every
        for seed in seeds:
            s = ot_solver(side, b0s[seed], precision, device)
            k = 0
            while True:
                xs.setdefault(side, []).append(s.cnn_inputs(norm).clone())
                r, d1 = s.ratio_fields(with_d1=True)
                ys.setdefault(side, []).append(r)
                ws.setdefault(side, []).append(flux_weights(d1))
                k += 1
                if max_snaps and k >= max_snaps:
                    break
                rc, done, t = s.advance_rc(every, t_end=t_end)
                if rc != sx.OK:
                    # the run left the physical range: the snapshots taken so far
                    # are of valid states; stop this run here
                    if log:
                        log(f"[data] side {side} seed {seed}: stopped at a non-physical state, t = {t:.3f}")
                    break
                if done < every or t >= t_end * (1 - 1e-12):
                    break
            if log:
                log(f"[data] side {side} seed {seed} b0x{b0s[seed]:.3f}: {k} snapshots, t = {s.diagnostics()['t']:.3f}")
            s.close()
    return Dataset(tuple(norm), {k: torch.stack(v) for k, v in xs.items()},
                   {k: torch.stack(v) for k, v in ys.items()}, {k: torch.stack(v) for k, v in ws.items()},
                   {"sides": list(sides), "seeds": list(seeds), "snap_every": snap_every if isinstance(snap_every, int)
                    else {int(k): int(v) for k, v in snap_every.items()}, "t_end": t_end,
                    "b0": b0s})


def train(net: Network, data: Dataset, iters: int, batch_pixels: int = 1 << 19, lr: float = 2e-3,
          lr_end: float = 2e-4, seed: int = 0, log=None, log_every: int = 100, weighted: bool = True) -> List[float]:
    """Adam on random mini-batches (whole periodic snapshots of one size per
    step, sizes visited in proportion to their pixel counts), cosine-decayed
    learning rate, flux-weighted loss by default.  Returns the loss history
    (every log_every steps)."""
    rng = np.random.default_rng(seed)
    sides = sorted(data.x)
    weights = np.array([data.x[s].shape[0] * s * s for s in sides], dtype=np.float64)
    weights /= weights.sum()
    hist = []
    for it in range(iters):
        side = sides[rng.choice(len(sides), p=weights)]
        m = data.x[side].shape[0]
        n = max(1, min(m, batch_pixels // (side * side)))
        idx = torch.as_tensor(rng.choice(m, size=n, replace=False), device=data.x[side].device)
        x = data.x[side].index_select(0, idx).contiguous()
        y = data.y[side].index_select(0, idx).contiguous()
        wt = data.w[side].index_select(0, idx).contiguous() if weighted else None
        f = 0.5 * (1 + math.cos(math.pi * it / max(1, iters - 1)))
        loss = net.train_step(x, y, lr_end + (lr - lr_end) * f, wt)
        if (it % log_every == 0) or it == iters - 1:
            v = float(loss.item())
            hist.append(v)
            if log:
                log(f"[train] it {it} side {side} n {n} loss {v:.3e}")
    return hist


def evaluate(net: Network, data: Dataset, max_images: int = 16, weighted: bool = True) -> float:
    """(Flux-weighted) mean squared error over (up to max_images evenly
    spaced) snapshots of every size, weighted by pixel count."""
    tot, cnt = 0.0, 0
    for side in sorted(data.x):
        m = data.x[side].shape[0]
        idx = np.unique(np.linspace(0, m - 1, min(m, max_images)).astype(np.int64))
        for i in idx:
            wt = data.w[side][i:i + 1] if weighted else None
            l = net.loss_of(data.x[side][i:i + 1], data.y[side][i:i + 1], wt)
            tot += l * side * side
            cnt += side * side
    return tot / cnt
