"""FP64 oracle of the learned noise-level network -- TEST INFRASTRUCTURE ONLY.

The paper estimates sigma with a CNN classifier (Sec. III-E-1, Fig. 5) whose
training data and weights are not available.  The library replaces it with a
small regression network that predicts log(sigma) per 8x8 block; this file
is the plain FP64 definition of that network, its loss and its gradients,
against which the GPU forward and backward kernels are checked.

Network (same definition as the library's kernels, written independently):
  input   x0 = (u8 - 128) / 64, NHWC, C = 1 or 3 channels
  layer 1 3x3 conv C->32, stride 2, zero padding 1, ReLU
  layer 2 3x3 conv 32->32, stride 2, padding 1, ReLU
  layer 3 3x3 conv 32->32, stride 2, padding 1, ReLU      (one output per 8x8 block)
  layer 4 3x3 conv 32->32, stride 1, padding 1, ReLU
  layer 5 3x3 conv 32->32, stride 1, padding 1, ReLU
  layer 6 3x3 conv 32->1,  stride 1, padding 1            -> z = log(sigma), sigma on 0..255
  loss    mean over blocks of |z - log(sigma_target)|
  update  Adam (adam_step) on FP32 master weights, bf16 copies for the forward pass
A convolution is y[n,yo,xo,co] = b[co] + sum_{ky,kx,ci} w[co,ky,kx,ci] * xpad[n, s*yo+ky, s*xo+kx, ci]
with xpad the input padded by one zero pixel on every side; Ho = ceil(H/s).
Parameters are flat FP32/FP64 in layer order, each layer w[co][ky][kx][ci] then b[co].
"""
from __future__ import annotations

import numpy as np

LAYERS = [(None, 32, 2, True), (32, 32, 2, True), (32, 32, 2, True), (32, 32, 1, True), (32, 32, 1, True),
          (32, 1, 1, False)]  # (ci, co, stride, relu); ci None = image channels


def layer_shapes(c: int):
    out = []
    for ci, co, s, relu in LAYERS:
        out.append((c if ci is None else ci, co, s, relu))
    return out


def n_params(c: int) -> int:
    return sum(co * 9 * ci + co for ci, co, _, _ in layer_shapes(c))


def unflatten(flat: np.ndarray, c: int):
    flat = np.asarray(flat, dtype=np.float64)
    params, off = [], 0
    for ci, co, s, relu in layer_shapes(c):
        w = flat[off:off + co * 9 * ci].reshape(co, 3, 3, ci)
        off += co * 9 * ci
        b = flat[off:off + co]
        off += co
        params.append((w, b))
    assert off == flat.size
    return params


def flatten(params) -> np.ndarray:
    return np.concatenate([np.concatenate([w.reshape(-1), b.reshape(-1)]) for w, b in params])


def conv_forward(x: np.ndarray, w: np.ndarray, b: np.ndarray, s: int) -> np.ndarray:
    n, H, W, ci = x.shape
    Ho, Wo = -(-H // s), -(-W // s)
    xp = np.zeros((n, H + 2 + 2 * s, W + 2 + 2 * s, ci))
    xp[:, 1:H + 1, 1:W + 1, :] = x
    y = np.zeros((n, Ho, Wo, w.shape[0])) + b
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + s * Ho:s, kx:kx + s * Wo:s, :]
            y += patch @ w[:, ky, kx, :].T
    return y


def conv_backward(x: np.ndarray, w: np.ndarray, s: int, dy: np.ndarray):
    """Gradients of conv_forward w.r.t. its input, weights and bias, given dL/dy."""
    n, H, W, ci = x.shape
    Ho, Wo = dy.shape[1], dy.shape[2]
    xp = np.zeros((n, H + 2 + 2 * s, W + 2 + 2 * s, ci))
    xp[:, 1:H + 1, 1:W + 1, :] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + s * Ho:s, kx:kx + s * Wo:s, :]
            dw[:, ky, kx, :] = np.einsum("nhwo,nhwi->oi", dy, patch)
            dxp[:, ky:ky + s * Ho:s, kx:kx + s * Wo:s, :] += dy @ w[:, ky, kx, :]
    db = dy.sum(axis=(0, 1, 2))
    return dxp[:, 1:H + 1, 1:W + 1, :], dw, db


def input_tensor(u8: np.ndarray) -> np.ndarray:
    a = np.asarray(u8)
    if a.ndim == 2:
        a = a[None, :, :, None]
    elif a.ndim == 3:
        a = a[None] if a.shape[2] in (1, 3) and a.shape[0] > 3 else a[..., None]
    return (a.astype(np.float64) - 128.0) / 64.0


def forward(flat: np.ndarray, u8_nhwc: np.ndarray, c: int, act_round=None):
    """z (N, Hb, Wb) and the activations; act_round, if given, is applied to every stored
    activation (used to mirror a lower-precision activation format)."""
    params = unflatten(flat, c)
    x = (np.asarray(u8_nhwc, dtype=np.float64) - 128.0) / 64.0
    acts = [x]
    for (w, b), (ci, co, s, relu) in zip(params, layer_shapes(c)):
        y = conv_forward(acts[-1], w, b, s)
        if relu:
            y = np.maximum(y, 0.0)
            if act_round is not None:
                y = act_round(y)
        acts.append(y)
    return acts[-1][..., 0], acts


def loss_and_grad(flat: np.ndarray, u8_nhwc: np.ndarray, target_log: np.ndarray, c: int, act_round=None):
    """Mean |z - target| and its gradient w.r.t. the flat parameters (subgradient 0 at ties)."""
    params = unflatten(flat, c)
    z, acts = forward(flat, u8_nhwc, c, act_round)
    diff = z - target_log
    loss = float(np.mean(np.abs(diff)))
    dz = np.sign(diff) / diff.size
    dy = dz[..., None]
    grads = []
    shapes = layer_shapes(c)
    for li in range(len(params) - 1, -1, -1):
        w, b = params[li]
        ci, co, s, relu = shapes[li]
        if relu:
            dy = dy * (acts[li + 1] > 0)
        dx, dw, db = conv_backward(acts[li], w, s, dy)
        grads.append((dw, db))
        dy = dx
    grads.reverse()
    return loss, flatten(grads)


def adam_step(w: np.ndarray, m: np.ndarray, v: np.ndarray, g: np.ndarray, t: int, lr: float, b1: float = 0.9,
              b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma and Ba, "Adam: A Method for Stochastic Optimization", ICLR 2015,
    Algorithm 1) in FP64, step number t >= 1: the biased first and second moment estimates are
    updated with the gradient g, corrected by 1 - b^t, and the parameters move by
    lr * m_hat / (sqrt(v_hat) + eps).  Returns the new (w, m, v)."""
    w, m, v, g = (np.asarray(a, dtype=np.float64) for a in (w, m, v, g))
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    return w - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def block_targets(sigma_field: np.ndarray, B: int = 8) -> np.ndarray:
    """Per-block label: log of the root-mean-square sigma over each BxB block (edge blocks partial)."""
    h, w = sigma_field.shape
    hb, wb = -(-h // B), -(-w // B)
    out = np.zeros((hb, wb))
    for i in range(hb):
        for j in range(wb):
            blk = sigma_field[i * B:(i + 1) * B, j * B:(j + 1) * B]
            out[i, j] = 0.5 * np.log(np.mean(blk * blk))
    return out
