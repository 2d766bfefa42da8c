"""Noise-level oracle (FP64, NumPy) -- TEST INFRASTRUCTURE ONLY.

* sigma_est per 128x128 sub-image: the paper obtains sigma_est from a CNN
  classifier (Sec. III-E-1, Fig. 5) trained on data that is not available.
  In its place this module takes the eigenvalues of the covariance of all
  overlapping 8x8 patches (the rationale is Eq. 12: noisy correlation =
  clean correlation + sigma^2 I) and picks the noise-only tail with the rule
  of Chen, Zhu and Heng, "An Efficient Statistical Method for Image Noise
  Level Estimation" (ICCV 2015): the first tail {lambda_i..lambda_m}
  (eigenvalues in descending order) whose mean is also its median, i.e. as
  many tail eigenvalues lie above the mean as below it; sigma^2 is that mean.
* The adjustment of Eq. 23 (Sec. III-E-1): for a few sampled groups per
  sub-image, the rank position a of the alternating eigenvalue (Eq. 22) among
  the K eigenvalues of circ(G) circ(G)^T (Eq. 15-16); a group votes
  "adjust" when a <= gamma; a majority of votes sets sigma = sigma_est/beta.

Readings (the paper is silent): sub-images are a non-overlapping 128x128
partition (edge tiles partial); a reference belongs to the tile holding its
top-left pixel; the covariance uses the patches whose top-left pixel lies in
the tile (clamped to the last valid position); 15 votes per tile drawn with
replacement by the counter-based SplitMix64 generator, or every reference
of a tile holding at most 15; the eigenvalues of the circulant Gram are its
closed-form spectrum lambda_k = |sum_m p_m exp(-2 pi i k m / K)|^2, each
counted with its multiplicity; eigenvalues within 1e-10*K*c_0 of the
alternating one count as equal to it.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def splitmix64(state: int) -> int:
    """One SplitMix64 output for the state after its increment (Steele, Lea,
    Flood 2014): z = state; z = (z ^ z>>30) * 0xBF58476D1CE4E5B9;
    z = (z ^ z>>27) * 0x94D049BB133111EB; z ^ z>>31."""
    z = state & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def tile_grid(h: int, w: int, T: int = 128):
    return (h + T - 1) // T, (w + T - 1) // T


def tile_of_refs(ys: np.ndarray, xs: np.ndarray, h: int, w: int, T: int = 128) -> np.ndarray:
    """Tile id (ty*ntx + tx) of every reference r = iy*nx + ix."""
    nty, ntx = tile_grid(h, w, T)
    ty = (ys // T)[:, None]
    tx = (xs // T)[None, :]
    return (ty * ntx + tx).reshape(-1).astype(np.int64)


def chen_tail_sigma2(eigs_desc: np.ndarray) -> float:
    """sigma^2 from eigenvalues sorted in descending order (Chen et al. 2015)."""
    lam = np.asarray(eigs_desc, dtype=np.float64)
    m = lam.size
    for i in range(m):
        tail = lam[i:]
        tau = tail.mean()
        if np.count_nonzero(tail > tau) == np.count_nonzero(tail < tau):
            return float(tau)
    return float(lam[-1])


def patch_covariance(plane: np.ndarray, y0: int, y1: int, x0: int, x1: int, ps: int = 8) -> np.ndarray:
    """Covariance (FP64) of the ps x ps patches with top-left in [y0,y1] x [x0,x1] of one uint8 plane.
    Sums are exact integers (< 2^53) before the division."""
    n = (y1 - y0 + 1) * (x1 - x0 + 1)
    cols = []
    for i in range(ps):
        for j in range(ps):
            cols.append(plane[y0 + i:y1 + i + 1, x0 + j:x1 + j + 1].reshape(-1))
    P = np.stack(cols, axis=1).astype(np.float64)  # n x ps^2
    s1 = P.sum(axis=0)
    s2 = P.T @ P
    return s2 / n - np.outer(s1, s1) / (n * n)


def sigma_est_tiles(img: np.ndarray, T: int = 128, ps: int = 8, tiles=None) -> np.ndarray:
    """Plain sigma_est per sub-image: sqrt(mean over channels of the Chen tail variance).
    With `tiles` (raster tile indices) only those entries are computed (the others are 0)."""
    a = img if img.ndim == 3 else img[:, :, None]
    h, w, c = a.shape
    nty, ntx = tile_grid(h, w, T)
    out = np.zeros(nty * ntx, dtype=np.float64)
    todo = range(nty * ntx) if tiles is None else sorted(set(int(t) for t in tiles))
    for t in todo:
        ty, tx = divmod(t, ntx)
        y0 = min(ty * T, h - ps)
        y1 = min(ty * T + T - 1, h - ps)
        x0 = min(tx * T, w - ps)
        x1 = min(tx * T + T - 1, w - ps)
        s2 = 0.0
        for ch in range(c):
            C = patch_covariance(a[:, :, ch], y0, y1, x0, x1, ps)
            ev = np.linalg.eigvalsh(C)[::-1]
            s2 += chen_tail_sigma2(ev)
        out[t] = np.sqrt(max(s2 / c, 0.0))
    return out


def circulant_spectrum(P: np.ndarray) -> np.ndarray:
    """Eigenvalues lambda_k, k = 0..K/2, of circ(G) circ(G)^T for a group given as
    P[K, n] (integer patch vectors in group order), from the exact int64
    autocorrelations c_d = sum_m p_m . p_{(m+d) mod K}: lambda_k = sum_d c_d cos(2 pi k d / K)."""
    P = np.asarray(P, dtype=np.int64)
    K = P.shape[0]
    cd = np.array([int(np.sum(P * np.roll(P, -d, axis=0))) for d in range(K)], dtype=np.int64)
    lam = np.zeros(K // 2 + 1, dtype=np.float64)
    for k in range(K // 2 + 1):
        acc = 0.0
        for d in range(K):
            acc += float(cd[d]) * np.cos(2.0 * np.pi * ((k * d) % K) / K)
        lam[k] = acc
    return lam, cd


def rank_position(P: np.ndarray) -> int:
    """Rank a (1-based, ascending) of the alternating eigenvalue (Eq. 22) among
    the K eigenvalues of circ(G)circ(G)^T, each pair lambda_k = lambda_{K-k}
    counted twice."""
    lam, cd = circulant_spectrum(P)
    K = np.asarray(P).shape[0]
    lam_hat = lam[K // 2]
    tol = 1e-10 * K * float(cd[0])
    a = 1
    if lam[0] < lam_hat - tol:
        a += 1
    for k in range(1, K // 2):
        if lam[k] < lam_hat - tol:
            a += 2
    return a


def vote_samples(tile_refs: np.ndarray, tile_id: int, n_vote: int = 15, seed: int = 0) -> np.ndarray:
    """References that vote for one tile: all of them when there are at most
    n_vote, else n_vote draws (with replacement) tile_refs[h mod n] with
    h = SplitMix64 output number tile_id*n_vote + i + 1 of the seed."""
    n = len(tile_refs)
    if n <= n_vote:
        return np.asarray(tile_refs)
    out = []
    for i in range(n_vote):
        ctr = tile_id * n_vote + i + 1
        hval = splitmix64((seed + ctr * GOLDEN) & MASK64)
        out.append(tile_refs[hval % n])
    return np.asarray(out)


def group_vectors(img: np.ndarray, idx_row: np.ndarray, ps: int = 8) -> np.ndarray:
    """Patch vectors (all channels) of one group, member-major, as int64."""
    a = img if img.ndim == 3 else img[:, :, None]
    h, w, c = a.shape
    out = []
    for lin in idx_row:
        y, x = divmod(int(lin), w)
        out.append(a[y:y + ps, x:x + ps, :].reshape(-1))
    return np.stack(out).astype(np.int64)


def sigma_hat_tiles(img: np.ndarray, idx: np.ndarray, sigma_est: np.ndarray, ps: int, s: int,
                    T: int = 128, n_vote: int = 15, seed: int = 0, beta: float = 1.2, gamma: int = 13,
                    return_votes: bool = False):
    """Eq. 23 per tile: sigma_hat = sigma_est/beta if most sampled groups have a <= gamma."""
    from . import ref_grid
    a = img if img.ndim == 3 else img[:, :, None]
    h, w, _ = a.shape
    ys, xs = ref_grid(h, ps, s), ref_grid(w, ps, s)
    tiles = tile_of_refs(ys, xs, h, w, T)
    nty, ntx = tile_grid(h, w, T)
    sig = np.asarray(sigma_est, dtype=np.float64).copy()
    votes = np.zeros(nty * ntx, dtype=np.int64)
    nvotes = np.zeros(nty * ntx, dtype=np.int64)
    ranks = {}
    for t in range(nty * ntx):
        refs = np.nonzero(tiles == t)[0]
        if refs.size == 0:
            continue
        sample = vote_samples(refs, t, n_vote, seed)
        yes = 0
        for r in sample:
            ar = rank_position(group_vectors(img, idx[r], ps))
            ranks.setdefault(t, []).append(ar)
            if ar <= gamma:
                yes += 1
        votes[t] = yes
        nvotes[t] = len(sample)
        if 2 * yes > len(sample):
            sig[t] = sig[t] / beta
    if return_votes:
        return sig, votes, nvotes, ranks
    return sig


def tau_per_ref(sigma_tiles: np.ndarray, h: int, w: int, ps: int, s: int, c: int, K: int, T: int = 128,
                mult: float | None = None) -> np.ndarray:
    """tau of every reference = sigma_hat of its tile * sqrt(2 ln(c K ps^2))."""
    from . import ref_grid, tau_multiplier
    ys, xs = ref_grid(h, ps, s), ref_grid(w, ps, s)
    tiles = tile_of_refs(ys, xs, h, w, T)
    m = tau_multiplier(c, K, ps) if mult is None else mult
    return np.asarray(sigma_tiles, dtype=np.float64)[tiles] * m


def band_sigma(cube: np.ndarray, T: int = 128, ps: int = 8) -> np.ndarray:
    """Band-wise noise levels of a cube (h, w, B) (Sec. IV-D): sigma_b is the mean, over the
    band's T x T sub-images, of the plain estimate sigma_est of the band alone."""
    return np.array([sigma_est_tiles(np.ascontiguousarray(cube[:, :, b]), T, ps).mean()
                     for b in range(cube.shape[2])])


def band_sigma_rule(sig: np.ndarray):
    """Sec. IV-D: sigma_mean is the mean band level; bands above 2 sigma_mean are severely
    contaminated and take the result filtered at the highest level, the others the result
    filtered at sigma_mean.  Returns (sigma_mean, sigma_max, severe mask)."""
    sig = np.asarray(sig, dtype=np.float64)
    mean = float(sig.mean())
    return mean, float(sig.max()), sig > 2.0 * mean
