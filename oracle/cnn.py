"""FP64 reference of the hyper-diffusion surrogate network -- TEST INFRASTRUCTURE ONLY.

A small convolutional network predicts, per cell, the ten hyper-diffusion
coefficient ratios R (x faces: rho~, eps~, v_x, v_y, B~_y; y faces: rho~,
eps~, v_x, v_y, B~_x) from six local fields.  Four 3x3 convolutions with
periodic padding, ReLU between them, and an output 4 sigmoid(z) (the exact
ratio is bounded by 0 <= R <= 4).  Plain numpy in FP64; a convolution is the
sum over the nine offsets of a channel contraction of the shifted input.

Used by the tests to check the GPU kernels' forward pass, gradients and
optimiser step; pinned by finite differences and exact special cases.

Precision: the network is specified with BF16 weights and FP32 accumulation.
With ``bf16=True`` the reference rounds (round-to-nearest-even) at exactly the
points where that arithmetic holds BF16 values: the weights, every hidden
activation (a layer's input) and every back-propagated gradient that enters
a product (the error signal of each layer).  Sums stay in FP64, so the only
remaining difference to an FP32-accumulating implementation is the order and
precision of the sums.
"""

from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

LAYERS = [(6, 32), (32, 32), (32, 32), (32, 10)]
OFFSETS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]   # row-major over the 3x3 window


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), via float32, returned as float64."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def shift(x: np.ndarray, dy: int, dx: int) -> np.ndarray:
    """out[c, i, j] = x[c, (i + dy) mod H, (j + dx) mod W] (periodic padding)."""
    return np.roll(x, shift=(-dy, -dx), axis=(1, 2))


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x (Cin, H, W), w (Cout, Cin, 3, 3), b (Cout,) -> (Cout, H, W);
    w[o, c, dy + 1, dx + 1] multiplies x[c, i + dy, j + dx]."""
    cout = w.shape[0]
    y = np.zeros((cout,) + x.shape[1:])
    for dy, dx in OFFSETS:
        y += np.einsum("oc,chw->ohw", w[:, :, dy + 1, dx + 1], shift(x, dy, dx))
    return y + b[:, None, None]


def conv3x3_grads(x: np.ndarray, w: np.ndarray, dy_: np.ndarray):
    """Gradients of sum(dy_ * conv3x3(x, w, b)) w.r.t. x, w and b."""
    dx_ = np.zeros_like(x)
    dw = np.zeros_like(w)
    for dy, dx in OFFSETS:
        xs = shift(x, dy, dx)
        dw[:, :, dy + 1, dx + 1] = np.einsum("ohw,chw->oc", dy_, xs)
        # y[o, p] += w[o, c] x[c, p + d]  =>  dx[c, q] += w[o, c] dy[o, q - d]
        dx_ += shift(np.einsum("oc,ohw->chw", w[:, :, dy + 1, dx + 1], dy_), -dy, -dx)
    db = dy_.sum(axis=(1, 2))
    return dx_, dw, db


def init_params(seed: int = 0) -> Dict[str, np.ndarray]:
    """He-style initialisation (seeded)."""
    rng = np.random.default_rng(seed)
    p = {}
    for l, (ci, co) in enumerate(LAYERS):
        p[f"w{l}"] = rng.normal(0.0, np.sqrt(2.0 / (9 * ci)), size=(co, ci, 3, 3))
        p[f"b{l}"] = np.zeros(co)
    return p


def _weights(p, l, bf16):
    w = p[f"w{l}"]
    return bf16_round(w) if bf16 else w


def forward(p: Dict[str, np.ndarray], x: np.ndarray, bf16: bool = False) -> Tuple[np.ndarray, List[np.ndarray]]:
    """Returns the predicted ratios 4 sigmoid(z4) and the cache for backward."""
    acts = [bf16_round(x) if bf16 else x]
    h = acts[0]
    for l in range(len(LAYERS)):
        z = conv3x3(h, _weights(p, l, bf16), p[f"b{l}"])
        if l < len(LAYERS) - 1:
            h = np.maximum(z, 0.0)
            if bf16:
                h = bf16_round(h)
        else:
            h = 4.0 / (1.0 + np.exp(-z))
        acts.append(h)
    return h, acts


def loss(pred: np.ndarray, target: np.ndarray, weight: np.ndarray = None) -> float:
    """Mean over all outputs of the (weighted) squared error."""
    w = 1.0 if weight is None else weight
    return float(np.mean(w * (pred - target) ** 2))


def backward(p: Dict[str, np.ndarray], acts: List[np.ndarray], target: np.ndarray,
             bf16: bool = False, count: int = 0, weight: np.ndarray = None) -> Dict[str, np.ndarray]:
    """Gradients of the (weighted) mean squared error w.r.t. every parameter.
    `count` is the number of outputs the mean runs over (default: this
    image's)."""
    pred = acts[-1]
    n = count if count else pred.size
    w = 1.0 if weight is None else weight
    g = 2.0 * w * (pred - target) / n
    # d(4 sigmoid(z))/dz = pred (1 - pred / 4)
    g = g * pred * (1.0 - pred / 4.0)
    grads = {}
    for l in reversed(range(len(LAYERS))):
        if bf16:
            g = bf16_round(g)
        h_in = acts[l]
        dx_, dw, db = conv3x3_grads(h_in, _weights(p, l, bf16), g)
        grads[f"w{l}"], grads[f"b{l}"] = dw, db
        if l > 0:
            g = dx_ * (acts[l] > 0.0)
    return grads


def batch_loss_and_grads(p, xs, ts, bf16: bool = False, ws=None):
    """(Weighted) mean squared error over a batch of images and its parameter gradients."""
    count = sum(t.size for t in ts)
    total = 0.0
    grads = {k: np.zeros_like(v) for k, v in p.items()}
    for i, (x, t) in enumerate(zip(xs, ts)):
        w = None if ws is None else ws[i]
        pred, acts = forward(p, x, bf16)
        total += float(np.sum((1.0 if w is None else w) * (pred - t) ** 2))
        g = backward(p, acts, t, bf16, count, w)
        for k in grads:
            grads[k] += g[k]
    return total / count, grads


def flatten(p) -> np.ndarray:
    """Parameter vector in the order w0, b0, w1, b1, w2, b2, w3, b3, each
    weight array row-major over (out channel, in channel, ky, kx)."""
    return np.concatenate([p[f"{a}{l}"].reshape(-1) for l in range(len(LAYERS)) for a in "wb"])


def unflatten(theta: np.ndarray) -> Dict[str, np.ndarray]:
    p, o = {}, 0
    for l, (ci, co) in enumerate(LAYERS):
        n = co * ci * 9
        p[f"w{l}"] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(co, ci, 3, 3)
        o += n
        p[f"b{l}"] = np.asarray(theta[o:o + co], dtype=np.float64).copy()
        o += co
    assert o == theta.size
    return p


NPARAM = sum(co * ci * 9 + co for ci, co in LAYERS)


def adam_step(p, grads, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), in place; t counts from 1."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * grads[k]
        v[k] = b2 * v[k] + (1 - b2) * grads[k] ** 2
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
