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


# ---- learned noise map -> thresholds (Sec. III-E-1, Eq. 22-23) ------------------------------
# The paper feeds a CNN's noise estimate into the thresholds and adjusts it per sub-image with
# the vote of Eq. 23.  Its CNN is not available; the library's network predicts z = log(sigma)
# for every 8x8 block instead.  The rule below is the reading the library implements:
#   judge   per 128 x 128 sub-image t, the mean learned sigma m_t over the blocks of t is kept
#           when sp_t / 1.5 <= m_t <= 1.5 sp_t (sp_t the plain estimate of t; m_t finite and
#           positive), otherwise the plain estimate stands for the tile: sigma_est_t = m_t or sp_t;
#   vote    Eq. 23 with sigma_est_t (votes from the tile's sampled groups): sigma_hat_t equals
#           sigma_est_t / beta on a majority, else sigma_est_t; the vote factor is their ratio;
#   block   the effective sigma of block b in tile t is exp(z_b) times the vote factor of t where
#           t kept the map, sigma_hat_t where it did not;
#   tau     a reference's threshold is the effective sigma of the block holding its top-left
#           pixel times sqrt(2 ln(c K ps^2)).
# A block lies in exactly one sub-image because 128 is a multiple of 8.

JUDGE_BOUND = 1.5


def blocks_of_tile(t: int, h: int, w: int, T: int = 128, B: int = 8):
    """Block rows and columns [by0, by1) x [bx0, bx1) of sub-image t (edge tiles partial)."""
    nty, ntx = tile_grid(h, w, T)
    ty, tx = divmod(t, ntx)
    hb, wb = -(-h // B), -(-w // B)
    bpt = T // B
    return ty * bpt, min(hb, (ty + 1) * bpt), tx * bpt, min(wb, (tx + 1) * bpt)


def judge_tile_sigma(block_sigma: np.ndarray, sp: float, bound: float = JUDGE_BOUND):
    """The judge on one tile given its blocks' learned sigma values: (sigma_est, use_plain).
    The mean is the correctly rounded sum (math.fsum) over the number of blocks."""
    import math
    v = np.asarray(block_sigma, dtype=np.float64).reshape(-1)
    mean = math.fsum(v.tolist()) / v.size if v.size else 0.0
    ok = math.isfinite(mean) and mean > 0.0 and sp > 0.0 and mean <= bound * sp and mean * bound >= sp
    return (mean, False) if ok else (float(sp), True)


def learned_judge(z: np.ndarray, sigma_plain: np.ndarray, h: int, w: int, T: int = 128,
                  bound: float = JUDGE_BOUND):
    """Per sub-image: (sigma_est, use_plain) of the learned map z (ceil(h/8) x ceil(w/8) log sigma)
    judged by the plain estimates sigma_plain."""
    z = np.asarray(z, dtype=np.float64)
    nty, ntx = tile_grid(h, w, T)
    se = np.zeros(nty * ntx)
    up = np.zeros(nty * ntx, dtype=bool)
    for t in range(nty * ntx):
        by0, by1, bx0, bx1 = blocks_of_tile(t, h, w, T)
        se[t], up[t] = judge_tile_sigma(np.exp(z[by0:by1, bx0:bx1]), float(sigma_plain[t]), bound)
    return se, up


def vote_factor(votes: np.ndarray, nvotes: np.ndarray, beta: float = 1.2) -> np.ndarray:
    """Eq. 23 as a factor per tile: 1/beta where most sampled groups voted "adjust", else 1."""
    votes, nvotes = np.asarray(votes), np.asarray(nvotes)
    return np.where(2 * votes > nvotes, 1.0 / beta, 1.0)


def effective_sigma_map(h: int, w: int, sigma_hat: np.ndarray, T: int = 128, z=None, use_plain=None,
                        factor=None) -> np.ndarray:
    """Effective sigma per 8x8 block (ceil(h/8) x ceil(w/8)): sigma_hat of the block's tile, or
    exp(z) of the block times the tile's vote factor where the tile kept the learned map."""
    nty, ntx = tile_grid(h, w, T)
    hb, wb = -(-h // 8), -(-w // 8)
    out = np.zeros((hb, wb))
    for t in range(nty * ntx):
        by0, by1, bx0, bx1 = blocks_of_tile(t, h, w, T)
        if z is None or use_plain[t]:
            out[by0:by1, bx0:bx1] = sigma_hat[t]
        else:
            out[by0:by1, bx0:bx1] = np.exp(np.asarray(z, dtype=np.float64)[by0:by1, bx0:bx1]) * factor[t]
    return out


def tau_from_sigma_map(smap: np.ndarray, h: int, w: int, ps: int, s: int, c: int, K: int,
                       mult: float | None = None) -> np.ndarray:
    """tau of every reference r = iy*nx + ix: the effective sigma of the block holding its
    top-left pixel times the multiplier."""
    from . import ref_grid, tau_multiplier
    ys, xs = ref_grid(h, ps, s), ref_grid(w, ps, s)
    m = tau_multiplier(c, K, ps) if mult is None else mult
    return (np.asarray(smap)[(ys // 8)[:, None], (xs // 8)[None, :]] * m).reshape(-1)


def thresholds(img: np.ndarray, ps: int, s: int, W: int, K: int, z=None, adaptive: bool = True, T: int = 128,
               n_vote: int = 15, seed: int = 0, beta: float = 1.2, gamma: int = 13, mult: float | None = None,
               sigma_known: float | None = None, tiles=None, sigma_plain=None, votes=None):
    """The noise-level rule on one image, from the pixels to the per-reference thresholds:
    sigma_est per sub-image (the known level, the plain estimate, or with a learned map z the
    judged level), the Eq. 23 vote on it (oracle groups of the sampled voters), the effective
    sigma per 8x8 block and tau per reference.  `tiles` restricts the work to those sub-images
    (entries of the others are NaN; references outside them get tau NaN).  sigma_plain (plain
    estimates per tile) and votes ((votes, nvotes) per tile, from groups of K members) may be
    passed in when already computed by this module for the same image.
    Returns a dict with sigma_plain, sigma_est, use_plain, votes, nvotes, sigma_hat, map, tau."""
    from . import block_match_list, ref_grid
    votes_given = votes
    a = img if img.ndim == 3 else img[:, :, None]
    h, w, c = a.shape
    nty, ntx = tile_grid(h, w, T)
    todo = list(range(nty * ntx)) if tiles is None else sorted(set(int(t) for t in tiles))
    nan = np.full(nty * ntx, np.nan)
    sp = nan.copy()
    if sigma_known is not None:
        sp[todo] = float(sigma_known)
    elif sigma_plain is not None:
        sp[todo] = np.asarray(sigma_plain, dtype=np.float64)[todo]
    else:
        sp[todo] = sigma_est_tiles(img, T, ps, tiles=todo)[todo]
    se, up = sp.copy(), np.zeros(nty * ntx, dtype=bool)
    if z is not None and sigma_known is None:
        zz = np.asarray(z, dtype=np.float64)
        for t in todo:
            by0, by1, bx0, bx1 = blocks_of_tile(t, h, w, T)
            se[t], up[t] = judge_tile_sigma(np.exp(zz[by0:by1, bx0:bx1]), float(sp[t]))
    votes = np.zeros(nty * ntx, dtype=np.int64)
    nvotes = np.zeros(nty * ntx, dtype=np.int64)
    if adaptive and votes_given is not None:
        votes[todo] = np.asarray(votes_given[0])[todo]
        nvotes[todo] = np.asarray(votes_given[1])[todo]
    elif adaptive:
        ys, xs = ref_grid(h, ps, s), ref_grid(w, ps, s)
        tile_of = tile_of_refs(ys, xs, h, w, T)
        for t in todo:
            refs = np.nonzero(tile_of == t)[0]
            if refs.size == 0:
                continue
            voters = vote_samples(refs, t, n_vote, seed)
            gi, _ = block_match_list(img, voters, ps, s, W, K)
            votes[t] = sum(rank_position(group_vectors(img, gi[i], ps)) <= gamma for i in range(len(voters)))
            nvotes[t] = len(voters)
    f = vote_factor(votes, nvotes, beta)
    sh = np.where(2 * votes > nvotes, se / beta, se)
    learned = z is not None and sigma_known is None
    smap = effective_sigma_map(h, w, sh, T, z=z if learned else None, use_plain=up, factor=f)
    for t in sorted(set(range(nty * ntx)) - set(todo)):
        by0, by1, bx0, bx1 = blocks_of_tile(t, h, w, T)
        smap[by0:by1, bx0:bx1] = np.nan
    tau = tau_from_sigma_map(smap, h, w, ps, s, c, K, mult)
    return {"sigma_plain": sp, "sigma_est": se, "use_plain": up, "votes": votes, "nvotes": nvotes,
            "sigma_hat": sh, "map": smap, "tau": tau}


def auto_group_size(sigma_ref: np.ndarray, cutoff: float) -> int:
    """Group size of an image in the batched auto mode (the library's reading: the K-selection
    of Sec. IV-A made per image): 16 when the mean effective sigma over its references, before the
    Eq. 23 vote, lies below the cutoff, else 32.  The vote then runs on groups of that size."""
    import math
    v = np.asarray(sigma_ref, dtype=np.float64).reshape(-1)
    return 16 if math.fsum(v.tolist()) / v.size < cutoff else 32


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
