"""Learns the shared ("globally-reused") t-SVD basis pair (U, V) -- run once,
writes the basis files the library and the oracle both read as input.

Sec. III-B (Eq. 10-11, Fig. 4, Table I): the paper learns one global pair
from all reference patches of one image and reuses it for every other
image.  Per Fourier slice f of the patches (DFT along the channel mode,
Eq. 5), U_hat^(f) holds the eigenvectors of C_row = sum P_hat P_hat^H and
V_hat^(f) those of C_col = sum P_hat^H P_hat, in descending eigenvalue
order.  The paper's source image (the first CC15 image) is not available; a
seeded clean synthetic 512x512 image (seed 0) stands in for it.

Eigenvectors are fixed only up to a unit phase; this script fixes it by
making the entry of largest modulus (the first one among equals) real and
positive.  Slices f and c-f are complex conjugates (so U and V are real).

Usage:  python -m oracle.learn_basis  [out_dir]
"""
from __future__ import annotations

import os
import sys

import numpy as np

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import synth  # noqa: E402


def _fix_phase(Q: np.ndarray) -> np.ndarray:
    Q = Q.copy()
    for j in range(Q.shape[1]):
        k = int(np.argmax(np.abs(Q[:, j])))
        ph = Q[k, j] / abs(Q[k, j])
        Q[:, j] = Q[:, j] * np.conj(ph)
        Q[k, j] = abs(Q[k, j])
    return Q


def _patches(img: np.ndarray, ps: int, stride: int) -> np.ndarray:
    """All reference patches of the grid of Algorithm 1, (n, ps, ps, c) FP64."""
    a = img if img.ndim == 3 else img[:, :, None]
    h, w, c = a.shape
    from oracle import ref_grid
    ys, xs = ref_grid(h, ps, stride), ref_grid(w, ps, stride)
    return np.stack([a[y:y + ps, x:x + ps, :] for y in ys for x in xs]).astype(np.float64)


def slice_covariances(img: np.ndarray, ps: int = 8, stride: int = 4):
    """Per Fourier slice f (Eq. 5 along the channel mode) of all reference patches P:
    C_row^(f) = sum P_hat P_hat^H and C_col^(f) = sum P_hat^H P_hat, as (c, ps, ps) complex."""
    ph = np.fft.fft(_patches(img, ps, stride), axis=3)
    c = ph.shape[3]
    Crow = np.zeros((c, ps, ps), dtype=np.complex128)
    Ccol = np.zeros((c, ps, ps), dtype=np.complex128)
    for f in range(c):
        P = ph[:, :, :, f]
        Crow[f] = np.einsum("nij,nkj->ik", P, np.conj(P))
        Ccol[f] = np.einsum("nji,njk->ik", np.conj(P), P)
    return Crow, Ccol


def channel_gram(img: np.ndarray, ps: int = 8, stride: int = 4) -> np.ndarray:
    """Exact integer sums over all reference patches P, (2, c, c, ps, ps) int64:
    [0][a][b][i][k] = sum_P sum_j P(i, j, a) P(k, j, b) (rows), [1][a][b][i][k] = sum_P sum_j
    P(j, i, a) P(j, k, b) (columns).  The slice covariances above are their combinations
    sum_ab w^(f(a-b)) [0][a][b] and sum_ab w^(f(b-a)) [1][a][b], w = exp(-2 pi i / c)."""
    P = _patches(img, ps, stride).astype(np.int64)
    row = np.einsum("nija,nkjb->abik", P, P)
    col = np.einsum("njia,njkb->abik", P, P)
    return np.stack([row, col])


def learn(img: np.ndarray, ps: int = 8, stride: int = 4):
    """Returns (U, V) as real (ps, ps, c) tensors learned from the reference patches of img."""
    a = img if img.ndim == 3 else img[:, :, None]
    c = a.shape[2]
    from oracle import from_slices
    Crow_all, Ccol_all = slice_covariances(img, ps, stride)
    Uh = np.zeros((c, ps, ps), dtype=np.complex128)
    Vh = np.zeros((c, ps, ps), dtype=np.complex128)
    for f in range(c):
        if f > c - f and c - f > 0:
            Uh[f] = np.conj(Uh[c - f])
            Vh[f] = np.conj(Vh[c - f])
            continue
        for C, dst in ((Crow_all[f], Uh), (Ccol_all[f], Vh)):
            C = 0.5 * (C + C.conj().T)
            ev, Q = np.linalg.eigh(C)
            Q = Q[:, ::-1]
            dst[f] = _fix_phase(Q)
        if 2 * f == c:  # real slice for even c
            Uh[f] = Uh[f].real
            Vh[f] = Vh[f].real
    U = np.real(np.fft.ifft(Uh, axis=0))
    V = np.real(np.fft.ifft(Vh, axis=0))
    return from_slices(U), from_slices(V)


def write_basis(path: str, U: np.ndarray, V: np.ndarray):
    from oracle import to_slices
    raw = np.concatenate([to_slices(U).reshape(-1), to_slices(V).reshape(-1)]).astype("<f8")
    raw.tofile(path)


def main(out_dir: str | None = None):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out_dir = out_dir or os.path.join(root, "paper_2512_23569_amd", "data")
    os.makedirs(out_dir, exist_ok=True)
    rgb = synth.make_clean(512, 512, 3, seed=0)
    gray = synth.make_clean(512, 512, 1, seed=0)
    for img, c in ((rgb, 3), (gray, 1)):
        U, V = learn(img)
        write_basis(os.path.join(out_dir, "basis_ps8_c%d.f64" % c), U, V)
        print("wrote basis_ps8_c%d.f64" % c)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else None)
