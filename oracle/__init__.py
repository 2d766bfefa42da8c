"""Haar-tSVD FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library and never calls
it.  The heavy loops (block matching, the per-group transform, aggregation)
live in ``htsvd_oracle.c`` (plain C, FP64, OpenMP over references); the
pieces below are plain NumPy in FP64.

Paper: "Image Denoising Using Global and Local Circulant Representation".
Sections cited per function.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "htsvd_oracle.c")
_LIB = os.path.join(_HERE, "_liborc.so")
_lib = None


def build(force: bool = False) -> str:
    """Compiles the C oracle with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i32, i64, dbl, p = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        lib.orc_ref_grid.argtypes = [i32, i32, i32, p]
        lib.orc_ref_count.argtypes = [i32, i32, i32]
        lib.orc_haar.argtypes = [i32, p]
        lib.orc_bcirc.argtypes = [p, i32, i32, p]
        lib.orc_patch_forward.argtypes = [p, p, i32, i32, p, p]
        lib.orc_patch_inverse.argtypes = [p, p, i32, i32, p, p]
        lib.orc_gcp_green.argtypes = [p, i64, i32, i32, i32, i32, i32, i32]
        lib.orc_block_match.argtypes = [p, i32, i32, i32, i64, i32, i32, i32, i32, i32, i32, p, p, i32]
        lib.orc_block_match_list.argtypes = [p, i32, i32, i32, i64, i32, i32, i32, i32, i32, i32, p, i64, p, p,
                                             i32]
        lib.orc_denoise.argtypes = [p, i32, i32, i32, i64, i32, i32, i32, i32, i32, i32, p, p, p, p, dbl, p,
                                    i32, i64, i64, p, p]
        lib.orc_filter_groups.argtypes = [p, i32, i32, i32, i64, i32, i32, i64, p, p, p, p, p, i32, p, p]
        lib.orc_block_match_video.argtypes = [p, i32, i32, i32, i32, i64, i32, i32, i32, i32, i32, i32, i32, p, p,
                                              i32]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    pass


def _check(code: int):
    if code != 0:
        raise OracleError({-1: "invalid argument", -2: "bad shape / too few candidates",
                           -3: "out of memory"}.get(code, str(code)))


def _img3(img: np.ndarray):
    a = np.ascontiguousarray(img, dtype=np.uint8)
    if a.ndim == 2:
        return a, a.shape[0], a.shape[1], 1
    return a, a.shape[0], a.shape[1], a.shape[2]


# ---- reference grid, Algorithm 1 ---------------------------------------------

def ref_grid(n: int, ps: int, s: int) -> np.ndarray:
    """Reference positions along one side: {0, s, 2s, ...} <= n-ps, plus n-ps."""
    out = np.zeros(n // s + 2, dtype=np.int32)
    cnt = _L().orc_ref_grid(n, ps, s, _ptr(out))
    return out[:cnt].copy()


# ---- Haar matrix, Sec. II-D (Eq. 7-8) ---------------------------------------

def haar(K: int) -> np.ndarray:
    H = np.zeros((K, K), dtype=np.float64)
    _check(_L().orc_haar(K, _ptr(H)))
    return H


# ---- t-product, Sec. II-C (Eq. 2-5) ------------------------------------------

def to_slices(T: np.ndarray) -> np.ndarray:
    """(ps, ps, c) -> slice-major (c, ps, ps) contiguous FP64."""
    return np.ascontiguousarray(np.moveaxis(np.asarray(T, dtype=np.float64), 2, 0))


def from_slices(S: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.moveaxis(S, 0, 2))


def bcirc(A: np.ndarray) -> np.ndarray:
    """bcirc of an (n, n, c) tensor, Eq. 2."""
    s = to_slices(A)
    c, n, _ = s.shape
    B = np.zeros((n * c, n * c), dtype=np.float64)
    _L().orc_bcirc(_ptr(s), n, c, _ptr(B))
    return B


def patch_forward(U: np.ndarray, V: np.ndarray, P: np.ndarray) -> np.ndarray:
    """S = U^T * P * V through bcirc products (Eq. 3, Eq. 19 without Haar). Tensors (ps, ps, c)."""
    u, v, p = to_slices(U), to_slices(V), to_slices(P)
    c, ps, _ = p.shape
    S = np.zeros_like(p)
    _check(_L().orc_patch_forward(_ptr(u), _ptr(v), ps, c, _ptr(p), _ptr(S)))
    return from_slices(S)


def patch_inverse(U: np.ndarray, V: np.ndarray, S: np.ndarray) -> np.ndarray:
    """P = U * S * V^T through bcirc products (Eq. 21 without Haar)."""
    u, v, s = to_slices(U), to_slices(V), to_slices(S)
    c, ps, _ = s.shape
    P = np.zeros_like(s)
    _check(_L().orc_patch_inverse(_ptr(u), _ptr(v), ps, c, _ptr(s), _ptr(P)))
    return from_slices(P)


def fft3(T: np.ndarray) -> np.ndarray:
    """DFT along the third mode (Eq. 5): T_hat^(f) = sum_k T^(k) exp(-2 pi i f k / c)."""
    return np.fft.fft(np.asarray(T, dtype=np.float64), axis=2)


def tprod_fft(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """t-product A*B computed slice-wise in the Fourier domain (Eq. 4)."""
    Ah, Bh = fft3(A), fft3(B)
    Ch = np.einsum("ijf,jkf->ikf", Ah, Bh)
    return np.real(np.fft.ifft(Ch, axis=2))


def ttranspose(A: np.ndarray) -> np.ndarray:
    """Tensor transpose: slice 0 transposed, slices 1..c-1 transposed in reverse order."""
    c = A.shape[2]
    out = np.empty((A.shape[1], A.shape[0], c), dtype=np.float64)
    out[:, :, 0] = A[:, :, 0].T
    for k in range(1, c):
        out[:, :, k] = A[:, :, c - k].T
    return out


def tau_multiplier(c: int, K: int, ps: int = 8) -> float:
    """tau = sigma * sqrt(2 log(c K ps^2)) (Sec. IV-A), natural log (Donoho's universal threshold)."""
    return float(np.sqrt(2.0 * np.log(c * K * ps * ps)))


# ---- grouping, Sec. III-A (Eq. 9) -------------------------------------------

def gcp_green(img: np.ndarray, y: int, x: int, ps: int = 8, gnum: int = 6, gden: int = 5) -> bool:
    a, h, w, c = _img3(img)
    return bool(_L().orc_gcp_green(_ptr(a), w * c, c, ps, y, x, gnum, gden))


def block_match(img: np.ndarray, ps: int, s: int, W: int, K: int, gnum: int = 6, gden: int = 5,
                nthreads: int = 0):
    """Groups of all references: (idx[n_ref, K] int32 with y*w+x, dist[n_ref, K] int64)."""
    a, h, w, c = _img3(img)
    L = _L()
    n_ref = L.orc_ref_count(h, ps, s) * L.orc_ref_count(w, ps, s)
    idx = np.zeros((n_ref, K), dtype=np.int32)
    dist = np.zeros((n_ref, K), dtype=np.int64)
    _check(L.orc_block_match(_ptr(a), h, w, c, w * c, ps, s, W, K, gnum, gden, _ptr(idx), _ptr(dist), nthreads))
    return idx, dist


def block_match_list(img: np.ndarray, refs, ps: int, s: int, W: int, K: int, gnum: int = 6, gden: int = 5,
                     nthreads: int = 0):
    """Groups of the listed references (raster indices into the reference grid), same rule
    as block_match: (idx[len(refs), K], dist[len(refs), K])."""
    a, h, w, c = _img3(img)
    L = _L()
    r = np.ascontiguousarray(np.asarray(refs, dtype=np.int64))
    idx = np.zeros((r.size, K), dtype=np.int32)
    dist = np.zeros((r.size, K), dtype=np.int64)
    _check(L.orc_block_match_list(_ptr(a), h, w, c, w * c, ps, s, W, K, gnum, gden, _ptr(r), r.size, _ptr(idx),
                                  _ptr(dist), nthreads))
    return idx, dist


# ---- denoising, Algorithm 1 ---------------------------------------------------

def denoise(img: np.ndarray, U: np.ndarray, V: np.ndarray, tau, ps: int = 8, s: int = 4, W: int = 21,
            K: int = 16, gnum: int = 6, gden: int = 5, guard: float = 0.0, nthreads: int = 0,
            r_begin: int = 0, r_end: int = -1, return_near: bool = False, pest=None, ra_on=None):
    """Haar-tSVD with per-reference thresholds (scalar tau = same for all).
    U, V: basis tensors (ps, ps, c).  Returns FP64 (h, w[, c]).
    pest (n_ref, c, ps, ps) FP64 and ra_on (n_ref,) bool: RA-Haar-tSVD (Eq. 24-25), the first
    Haar row of each flagged group replaced by sqrt(K) U^T * pest * V and not thresholded."""
    a, h, w, c = _img3(img)
    L = _L()
    n_ref = L.orc_ref_count(h, ps, s) * L.orc_ref_count(w, ps, s)
    tau_ref = np.ascontiguousarray(np.broadcast_to(np.asarray(tau, dtype=np.float64), (n_ref,)))
    u, v = to_slices(U), to_slices(V)
    out = np.zeros((h, w, c), dtype=np.float64)
    near = ctypes.c_int64(0)
    pe = ro = None
    if pest is not None:
        pe = np.ascontiguousarray(np.asarray(pest, dtype=np.float64).reshape(n_ref, c * ps * ps))
        ro = np.ascontiguousarray(np.broadcast_to(np.asarray(True if ra_on is None else ra_on, dtype=np.uint8),
                                                  (n_ref,)))
    _check(L.orc_denoise(_ptr(a), h, w, c, w * c, ps, s, W, K, gnum, gden, _ptr(tau_ref), _ptr(u), _ptr(v),
                         _ptr(out), float(guard), ctypes.byref(near), nthreads, r_begin, r_end,
                         None if pe is None else _ptr(pe), None if ro is None else _ptr(ro)))
    res = out[:, :, 0] if img.ndim == 2 else out
    return (res, int(near.value)) if return_near else res


def filter_groups(img: np.ndarray, idx: np.ndarray, U: np.ndarray, V: np.ndarray, tau, ps: int = 8,
                  nthreads: int = 0, pest=None, ra_on=None) -> np.ndarray:
    """Eq. 19-21 and uniform aggregation of the given groups idx (n_ref, K) of y*w + x, any channel
    count (hyperspectral tube patches, Sec. IV-D; the stacked frames of a video, Sec. IV-C).
    U, V: (ps, ps, c).  pest / ra_on: RA-Haar-tSVD as in denoise.  Returns FP64 (h, w, c)."""
    a = img if img.ndim == 3 else img[:, :, None]
    a = np.ascontiguousarray(a)
    h, w, c = a.shape
    ix = np.ascontiguousarray(idx, dtype=np.int32)
    n_ref, K = ix.shape
    tau_ref = np.ascontiguousarray(np.broadcast_to(np.asarray(tau, dtype=np.float64), (n_ref,)))
    u, v = to_slices(U), to_slices(V)
    out = np.zeros((h, w, c), dtype=np.float64)
    pe = ro = None
    if pest is not None:
        pe = np.ascontiguousarray(np.asarray(pest, dtype=np.float64).reshape(n_ref, c * ps * ps))
        ro = np.ascontiguousarray(np.broadcast_to(np.asarray(True if ra_on is None else ra_on, dtype=np.uint8),
                                                  (n_ref,)))
    _check(_L().orc_filter_groups(_ptr(a), h, w, c, w * c, ps, K, n_ref, _ptr(ix), _ptr(tau_ref), _ptr(u), _ptr(v),
                                  _ptr(out), nthreads, None if pe is None else _ptr(pe),
                                  None if ro is None else _ptr(ro)))
    return out


def block_match_video(frames: np.ndarray, ps: int, s: int, W: int, K: int, radius: int, gnum: int = 6,
                      gden: int = 5, nthreads: int = 0):
    """Spatio-temporal groups of a video (T, h, w[, c]) (Sec. IV-C): (idx[T*ny*nx, K] int32 of
    (f*h + y)*w + x in the frames stacked vertically, dist int64)."""
    v = np.ascontiguousarray(frames if frames.ndim == 4 else frames[..., None])
    T, h, w, c = v.shape
    L = _L()
    n_ref = T * L.orc_ref_count(h, ps, s) * L.orc_ref_count(w, ps, s)
    idx = np.zeros((n_ref, K), dtype=np.int32)
    dist = np.zeros((n_ref, K), dtype=np.int64)
    _check(L.orc_block_match_video(_ptr(v), T, h, w, c, w * c, ps, s, W, K, radius, gnum, gden, _ptr(idx), _ptr(dist),
                                   nthreads))
    return idx, dist


def band_guide(cube: np.ndarray) -> np.ndarray:
    """Grouping image of a hyperspectral cube (h, w, bands): the band mean rounded half up,
    (sum + bands // 2) // bands, exact in integers."""
    b = cube.shape[2]
    return ((cube.astype(np.int64).sum(axis=2) + b // 2) // b).astype(np.uint8)


def n_refs(h: int, w: int, ps: int, s: int):
    L = _L()
    return L.orc_ref_count(h, ps, s), L.orc_ref_count(w, ps, s)


# ---- basis files ---------------------------------------------------------------

def load_basis(path: str, ps: int, c: int):
    """A basis file holds U then V, each ps*ps*c little-endian FP64, slice-major."""
    raw = np.fromfile(path, dtype="<f8")
    n = ps * ps * c
    if raw.size != 2 * n:
        raise OracleError("basis file has %d values, expected %d" % (raw.size, 2 * n))
    U = from_slices(raw[:n].reshape(c, ps, ps))
    V = from_slices(raw[n:].reshape(c, ps, ps))
    return U, V


from .estimator import (sigma_est_tiles, chen_tail_sigma2, circulant_spectrum, rank_position,  # noqa: E402
                        vote_samples, sigma_hat_tiles, splitmix64, tile_of_refs, tau_per_ref, band_sigma,
                        band_sigma_rule, learned_judge, thresholds, effective_sigma_map,
                        tau_from_sigma_map, auto_group_size)
