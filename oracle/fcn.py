"""Refinement network of RA-Haar-tSVD in FP64 (test infrastructure: only tests, the smoke check
and the benchmark's CPU baseline use this module).

Sec. III-E-2 (Eq. 24-25): the first row of the group's Haar projection is sqrt(K) times
the group's mean patch; a plain fully connected network (as in Burger et al.) maps the noisy
mean patch to a cleaner one, trained by residual learning on mean patches of noisy/clean
groups, and applied where the noise level exceeds 30 (Sec. IV-B).  The paper gives neither the
layer sizes nor the input scaling; this is the reading used throughout (the GPU network has the
same definition):

    x     = (p - 128) / 128              p: mean patch, P = 64c values, slice-major (c, 8, 8)
    h1    = relu(W1 x + b1)              W1: H x P
    h2    = relu(W2 h1 + b2)             W2: H x H
    r     = W3 h2 + b3                   W3: P x H
    p_est = p - 128 r                    (r estimates the noise of the mean, scaled)

with H = 256 for c = 3 and H = 128 for c = 1.  Parameters are flattened as W1, b1, W2, b2,
W3, b3, each row-major.  Training minimises the mean over samples and entries of
(r - r*)^2, r* = (p_noisy - p_clean) / 128.
"""
from __future__ import annotations

import numpy as np

SCALE = 128.0


def hidden(c: int) -> int:
    return 256 if c == 3 else 128


def shapes(c: int):
    P, H = 64 * c, hidden(c)
    return [(H, P), (H,), (H, H), (H,), (P, H), (P,)]


def param_count(c: int) -> int:
    return int(sum(np.prod(s) for s in shapes(c)))


def unflatten(params: np.ndarray, c: int):
    out, o = [], 0
    for s in shapes(c):
        n = int(np.prod(s))
        out.append(np.asarray(params[o:o + n], dtype=np.float64).reshape(s))
        o += n
    if o != params.size:
        raise ValueError("expected %d parameters, got %d" % (o, params.size))
    return out


def init_params(c: int, seed: int) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases, from a seeded PCG64 stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for s in shapes(c):
        if len(s) == 2:
            bound = np.sqrt(6.0 / s[1])
            parts.append(rng.uniform(-bound, bound, s).reshape(-1))
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts)


def forward(params: np.ndarray, means: np.ndarray, c: int, return_hidden: bool = False):
    """means: (N, P) noisy mean patches (0..255 scale).  Returns r (N, P) (and the hidden
    activations); the refined mean is means - 128 r."""
    W1, b1, W2, b2, W3, b3 = unflatten(params, c)
    x = (np.asarray(means, dtype=np.float64) - SCALE) / SCALE
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    r = h2 @ W3.T + b3
    if return_hidden:
        return r, (x, z1, h1, z2, h2)
    return r


def refine(params: np.ndarray, means: np.ndarray, c: int) -> np.ndarray:
    """Eq. 25: the refined mean patches p_est = p - 128 r."""
    return np.asarray(means, dtype=np.float64) - SCALE * forward(params, means, c)


def loss_and_grad(params: np.ndarray, noisy_means: np.ndarray, clean_means: np.ndarray, c: int):
    """Mean squared error of r against r* = (noisy - clean) / 128 and its gradient (backprop)."""
    W1, b1, W2, b2, W3, b3 = unflatten(params, c)
    r, (x, z1, h1, z2, h2) = forward(params, noisy_means, c, return_hidden=True)
    target = (np.asarray(noisy_means, dtype=np.float64) - np.asarray(clean_means, dtype=np.float64)) / SCALE
    n = r.size
    d = r - target
    loss = float(np.sum(d * d) / n)
    gr = 2.0 * d / n
    gW3 = gr.T @ h2
    gb3 = gr.sum(0)
    gh2 = gr @ W3
    gz2 = gh2 * (z2 > 0)
    gW2 = gz2.T @ h1
    gb2 = gz2.sum(0)
    gh1 = gz2 @ W2
    gz1 = gh1 * (z1 > 0)
    gW1 = gz1.T @ x
    gb1 = gz1.sum(0)
    return loss, np.concatenate([g.reshape(-1) for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def group_means(img: np.ndarray, idx: np.ndarray, ps: int = 8) -> np.ndarray:
    """Mean patch of every group: idx (n_ref, K) linear top-left positions y*w + x.  Returns
    (n_ref, c, ps, ps) FP64 (exact: sums of integers over a power-of-two K)."""
    a = img if img.ndim == 3 else img[:, :, None]
    h, w, c = a.shape
    n_ref, K = idx.shape
    out = np.zeros((n_ref, c, ps, ps))
    af = a.astype(np.float64)
    for k in range(K):
        ys, xs = idx[:, k] // w, idx[:, k] % w
        for i in range(ps):
            for j in range(ps):
                out[:, :, i, j] += af[ys + i, xs + j, :]
    return out / K
