"""Seeded synthetic inputs shared by the oracle, the tests, the benchmark and
the sigma-network training data.

This module draws random images and noise and nothing else: it holds none of
the denoiser's arithmetic (no block matching, no transform, no threshold, no
noise estimation).  Every function is a pure function of its seed.

The paper evaluates on real sRGB photographs (Kodak, SIDD, CC15, ...) that are
not available here; these generators stand in for them with the shapes and
noise levels the paper uses (8-bit RGB, sigma 5..75, 128x128 sub-images).

Clean gray layer, painted in this order (float64, 0..255 scale):
  1. a smooth gradient  a + b*x/W + c*y/H,  a~U[60,180], b,c~U[-40,40];
  2. 20 shapes, each an ellipse or a rectangle with probability 1/2, centre
     uniform in the image, half-axes U[0.03,0.25]*min(H,W), angle U[0,pi),
     flat intensity U[30,220] (painted over what is below);
  3. 3 sinusoidal gratings, period U[4,16] px, random orientation and phase,
     amplitude U[15,40], added inside a random disc of radius
     U[0.1,0.2]*min(H,W);
  4. optionally a 1/f-spectrum Gaussian texture normalised to std 10.
RGB images mix three independent gray layers with a random 3x3 matrix whose
rows are 0.5*e_i + 0.5*Dirichlet(1,1,1) (each row sums to 1), then clip to
[0,255] and round half-to-even.  Hyperspectral cubes (make_hsi) use gray layers
as abundances of a few smooth endmember spectra.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gray_layer", "make_clean", "make_hsi", "add_awgn", "add_poisson_gaussian",
    "smooth_sigma_field", "add_sigma_field_noise", "psnr", "make_cfg",
    "BATCH_SIZES", "batch_specs", "block_log_sigma", "sigma_crop",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def gray_layer(h: int, w: int, rng: np.random.Generator, texture: bool = False) -> np.ndarray:
    """One clean gray layer, float64 (h, w), before clipping/rounding."""
    yy = np.arange(h, dtype=np.float64)[:, None]
    xx = np.arange(w, dtype=np.float64)[None, :]
    a = rng.uniform(60, 180)
    b = rng.uniform(-40, 40)
    c = rng.uniform(-40, 40)
    img = a + b * xx / w + c * yy / h
    img = np.broadcast_to(img, (h, w)).copy()
    m = min(h, w)
    for _ in range(20):
        is_ellipse = rng.uniform() < 0.5
        cy = rng.uniform(0, h)
        cx = rng.uniform(0, w)
        ra = rng.uniform(0.03, 0.25) * m
        rb = rng.uniform(0.03, 0.25) * m
        ang = rng.uniform(0, np.pi)
        val = rng.uniform(30, 220)
        r = max(ra, rb) * 1.5 + 2
        y0, y1 = max(0, int(cy - r)), min(h, int(cy + r) + 1)
        x0, x1 = max(0, int(cx - r)), min(w, int(cx + r) + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        dy = yy[y0:y1] - cy
        dx = xx[:, x0:x1] - cx
        ca, sa = np.cos(ang), np.sin(ang)
        u = dx * ca + dy * sa
        v = -dx * sa + dy * ca
        if is_ellipse:
            mask = (u / ra) ** 2 + (v / rb) ** 2 <= 1.0
        else:
            mask = (np.abs(u) <= ra) & (np.abs(v) <= rb)
        sub = img[y0:y1, x0:x1]
        sub[mask] = val
    for _ in range(3):
        period = rng.uniform(4, 16)
        theta = rng.uniform(0, np.pi)
        phase = rng.uniform(0, 2 * np.pi)
        amp = rng.uniform(15, 40)
        cy = rng.uniform(0, h)
        cx = rng.uniform(0, w)
        rad = rng.uniform(0.1, 0.2) * m
        y0, y1 = max(0, int(cy - rad)), min(h, int(cy + rad) + 1)
        x0, x1 = max(0, int(cx - rad)), min(w, int(cx + rad) + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        dy = yy[y0:y1] - cy
        dx = xx[:, x0:x1] - cx
        mask = dx * dx + dy * dy <= rad * rad
        wave = amp * np.sin(2 * np.pi * (xx[:, x0:x1] * np.cos(theta) + yy[y0:y1] * np.sin(theta)) / period + phase)
        sub = img[y0:y1, x0:x1]
        sub[mask] += np.broadcast_to(wave, mask.shape)[mask]
    if texture:
        fy = np.fft.fftfreq(h)[:, None]
        fx = np.fft.rfftfreq(w)[None, :]
        f = np.sqrt(fy * fy + fx * fx)
        f[0, 0] = 1.0
        spec = (rng.standard_normal((h, w // 2 + 1)) + 1j * rng.standard_normal((h, w // 2 + 1))) / f
        spec[0, 0] = 0.0
        tex = np.fft.irfft2(spec, s=(h, w))
        sd = tex.std()
        if sd > 0:
            img += tex * (10.0 / sd)
    return img


def _quantise(x: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.rint(np.clip(x, 0.0, 255.0)).astype(np.uint8))


def make_clean(h: int, w: int, c: int, seed: int, texture: bool = False) -> np.ndarray:
    """Clean uint8 image, shape (h, w) for c=1, (h, w, 3) for c=3."""
    rng = _rng(seed)
    if c == 1:
        return _quantise(gray_layer(h, w, rng, texture))
    if c != 3:
        raise ValueError("c must be 1 or 3")
    layers = np.stack([gray_layer(h, w, rng, texture) for _ in range(3)], axis=0)
    mix = 0.5 * np.eye(3) + 0.5 * rng.dirichlet(np.ones(3), size=3)
    rgb = np.einsum("ij,jhw->hwi", mix, layers)
    return _quantise(rgb)


def make_hsi(h: int, w: int, bands: int, seed: int, n_end: int = 4) -> np.ndarray:
    """Clean uint8 hyperspectral cube (h, w, bands): n_end gray layers (as for make_clean) used
    as abundances, normalised to sum to 1 per pixel, times n_end smooth endmember spectra
    s_e(b) = 0.5 + 0.35 sin(2 pi (f_e b / bands + phi_e)) + 0.15 b / bands, f_e U[0.3, 1.5],
    phi_e U[0, 1), scaled by 255, rounded half-to-even and clipped."""
    rng = _rng(seed)
    ab = np.stack([gray_layer(h, w, rng, texture=bool(e % 2)) for e in range(n_end)], axis=2)
    ab = np.maximum(ab, 1.0)
    ab /= ab.sum(axis=2, keepdims=True)
    bb = np.arange(bands, dtype=np.float64) / bands
    spec = np.stack([0.5 + 0.35 * np.sin(2 * np.pi * (rng.uniform(0.3, 1.5) * bb + rng.uniform())) + 0.15 * bb
                     for _ in range(n_end)])
    return _quantise(255.0 * np.einsum("hwe,eb->hwb", ab, spec))


def make_video(T: int, h: int, w: int, c: int, seed: int, step: int = 2) -> np.ndarray:
    """Clean uint8 frames (T, h, w[, c]) of a scene in motion: a static background (make_clean of
    a larger canvas, textured) seen through a window that pans by up to `step` pixels per frame
    in each direction (a seeded random walk), with a textured object that moves on its own
    path across it."""
    rng = _rng(seed)
    pad = step * T + 8
    canvas = make_clean(h + 2 * pad, w + 2 * pad, c, seed, texture=True)
    obj = make_clean(h // 3 + 8, w // 3 + 8, c, seed + 1, texture=True)
    oy, ox = float(rng.uniform(0, h - obj.shape[0])), float(rng.uniform(0, w - obj.shape[1]))
    vy, vx = rng.uniform(-1.5, 1.5, 2) * step
    y, x = pad, pad
    frames = []
    for _ in range(T):
        f = canvas[y:y + h, x:x + w].copy()
        iy = int(np.clip(round(oy), 0, h - obj.shape[0]))
        ix = int(np.clip(round(ox), 0, w - obj.shape[1]))
        f[iy:iy + obj.shape[0], ix:ix + obj.shape[1]] = obj
        frames.append(f)
        y = int(np.clip(y + rng.integers(-step, step + 1), 0, 2 * pad))
        x = int(np.clip(x + rng.integers(-step, step + 1), 0, 2 * pad))
        oy, ox = oy + vy, ox + vx
    return np.ascontiguousarray(np.stack(frames))


def add_awgn(clean: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    """clean + N(0, sigma^2) in float, rounded half-to-even and clipped to uint8."""
    rng = _rng(seed)
    noisy = clean.astype(np.float64) + sigma * rng.standard_normal(clean.shape)
    return _quantise(noisy)


def add_band_awgn(cube: np.ndarray, sigmas, seed: int) -> np.ndarray:
    """Gaussian noise of level sigmas[b] on band b of a cube (h, w, B), rounded half-to-even and
    clipped to uint8 (non-uniform noise across bands)."""
    rng = _rng(seed)
    s = np.asarray(sigmas, dtype=np.float64).reshape(1, 1, -1)
    return _quantise(cube.astype(np.float64) + s * rng.standard_normal(cube.shape))


def add_poisson_gaussian(clean: np.ndarray, gain: float, read_sigma: float, seed: int) -> np.ndarray:
    """Signal-dependent noise on the 0..1 scale: y = gain*Poisson(x/gain) + N(0, (read/255)^2).

    With gain 0.01 and read sigma 8 (on 0..255) the variance on the 0..255 scale is
    2.55*x + 64.
    """
    rng = _rng(seed)
    x = clean.astype(np.float64) / 255.0
    y = gain * rng.poisson(x / gain) + (read_sigma / 255.0) * rng.standard_normal(clean.shape)
    return _quantise(y * 255.0)


def smooth_sigma_field(h: int, w: int, rng: np.random.Generator, lo: float = 5.0, hi: float = 75.0,
                       grid: int = 4) -> np.ndarray:
    """A smooth per-pixel sigma field: a grid x grid array of U[lo,hi] values,
    bilinearly upsampled (align-corners) to (h, w)."""
    g = rng.uniform(lo, hi, size=(grid, grid))
    ys = np.linspace(0, grid - 1, h)
    xs = np.linspace(0, grid - 1, w)
    y0 = np.clip(np.floor(ys).astype(int), 0, grid - 2)
    x0 = np.clip(np.floor(xs).astype(int), 0, grid - 2)
    ty = (ys - y0)[:, None]
    tx = (xs - x0)[None, :]
    g00 = g[y0][:, x0]
    g01 = g[y0][:, x0 + 1]
    g10 = g[y0 + 1][:, x0]
    g11 = g[y0 + 1][:, x0 + 1]
    return (1 - ty) * ((1 - tx) * g00 + tx * g01) + ty * ((1 - tx) * g10 + tx * g11)


def add_sigma_field_noise(clean: np.ndarray, sigma_field: np.ndarray, seed: int) -> np.ndarray:
    """clean + N(0, sigma(y,x)^2) per pixel (same sigma for every channel)."""
    rng = _rng(seed)
    s = sigma_field if clean.ndim == 2 else sigma_field[..., None]
    noisy = clean.astype(np.float64) + s * rng.standard_normal(clean.shape)
    return _quantise(noisy)


def psnr(ref: np.ndarray, est: np.ndarray) -> float:
    """PSNR in dB on the 0..255 scale; the estimate is clipped to [0,255] first."""
    a = ref.astype(np.float64)
    b = np.clip(np.asarray(est, dtype=np.float64), 0.0, 255.0)
    mse = np.mean((a - b) ** 2)
    if mse == 0:
        return float("inf")
    return float(10.0 * np.log10(255.0 ** 2 / mse))


# Workloads -----------------------------------------------------------------
# name -> (h, w, c, seed, texture, noise spec, params)
_CFGS = {
    "gray256_awgn25": dict(h=256, w=256, c=1, seed=1, texture=False, noise=("awgn", 25.0),
                           params=dict(stride=4, window=21, K=16, sigma=25.0, adaptive=0)),
    "rgb512_awgn50": dict(h=512, w=512, c=3, seed=2, texture=False, noise=("awgn", 50.0),
                          params=dict(stride=4, window=31, K=32, sigma=50.0, adaptive=1)),
    "rgb12mp_pg": dict(h=3000, w=4000, c=3, seed=3, texture=True, noise=("pg", 0.01, 8.0),
                       params=dict(stride=3, window=31, K=32, sigma=None, adaptive=1)),
}


def make_cfg(name: str, h: int | None = None, w: int | None = None):
    """Returns (clean, noisy, spec) for a named workload; h/w override the size
    (same generator, used for reduced samples)."""
    spec = dict(_CFGS[name])
    hh = spec["h"] if h is None else h
    ww = spec["w"] if w is None else w
    clean = make_clean(hh, ww, spec["c"], spec["seed"], spec["texture"])
    nz = spec["noise"]
    if nz[0] == "awgn":
        noisy = add_awgn(clean, nz[1], spec["seed"] + 1000)
    else:
        noisy = add_poisson_gaussian(clean, nz[1], nz[2], spec["seed"] + 1000)
    spec["h"], spec["w"] = hh, ww
    return clean, noisy, spec


BATCH_SIZES = [(256, 256), (384, 512), (768, 1024), (1080, 1920), (1536, 2048)]


def batch_specs(n: int = 64, seed: int = 4):
    """Per-image (h, w, sigma, seed) for the uneven batch: sizes uniform over
    BATCH_SIZES, AWGN sigma uniform in [5,75]."""
    rng = _rng(seed)
    out = []
    for i in range(n):
        h, w = BATCH_SIZES[int(rng.integers(0, len(BATCH_SIZES)))]
        sigma = float(rng.uniform(5.0, 75.0))
        out.append((h, w, sigma, seed + 1 + i))
    return out


def block_log_sigma(sigma_field: np.ndarray, B: int = 8) -> np.ndarray:
    """Training label of the sigma network: log of the root-mean-square sigma of every BxB
    block of a per-pixel sigma field (edge blocks partial)."""
    h, w = sigma_field.shape
    hb, wb = -(-h // B), -(-w // B)
    pad = np.zeros((hb * B, wb * B))
    cnt = np.zeros((hb * B, wb * B))
    pad[:h, :w] = sigma_field ** 2
    cnt[:h, :w] = 1.0
    s = pad.reshape(hb, B, wb, B).sum(axis=(1, 3))
    n = cnt.reshape(hb, B, wb, B).sum(axis=(1, 3))
    return 0.5 * np.log(s / n)


def sigma_crop(seed: int, size: int = 128, c: int = 3, lo: float = 5.0, hi: float = 75.0):
    """One training crop: a clean synthetic image with noise of a smooth random sigma field
    (4x4 grid of U[lo,hi] values, bilinear), and its per-8x8-block log-sigma label."""
    rng = _rng(seed)
    field = smooth_sigma_field(size, size, rng, lo, hi)
    clean = make_clean(size, size, c, int(rng.integers(0, 2 ** 31)))
    noisy = add_sigma_field_noise(clean, field, int(rng.integers(0, 2 ** 31)))
    return noisy, block_log_sigma(field).astype(np.float32), clean
