"""Shared test helpers (comparison metrics, input builders).  No method arithmetic."""
import numpy as np

import synth

# Parity bar for denoised pixels: at least 99.99% of the values within 1e-2 (0..255 scale)
# and |PSNR difference| <= 0.01 dB.
PIX_TOL = 1e-2
PIX_FRAC = 0.9999
PSNR_TOL = 0.01


def pixel_parity(gpu: np.ndarray, ref: np.ndarray, clean: np.ndarray | None = None):
    d = np.abs(gpu.astype(np.float64) - ref.astype(np.float64))
    frac = float(np.mean(d <= PIX_TOL))
    out = {"frac_within": frac, "max_abs": float(d.max()), "n_bad": int(np.sum(d > PIX_TOL))}
    if clean is not None:
        out["psnr_gpu"] = synth.psnr(clean, gpu)
        out["psnr_ref"] = synth.psnr(clean, ref)
        out["dpsnr"] = abs(out["psnr_gpu"] - out["psnr_ref"])
    return out


def assert_pixel_parity(gpu, ref, clean=None):
    m = pixel_parity(gpu, ref, clean)
    assert m["frac_within"] >= PIX_FRAC, m
    if clean is not None:
        assert m["dpsnr"] <= PSNR_TOL, m
    return m


def tie_heavy_image(h, w, c, seed):
    """Few gray levels, flat and saturated regions, a planted duplicate patch."""
    rng = np.random.default_rng(seed)
    shape = (h, w, c) if c == 3 else (h, w)
    img = (rng.integers(0, 4, shape) * 60).astype(np.uint8)
    img[: h // 5] = 0
    img[-(h // 6):, -(w // 4):] = 255
    if h >= 24 and w >= 24:
        img[12:20, 10:18] = img[0:8, 14:22]
    return img
