"""Trains the RA-Haar-tSVD refinement network (Sec. III-E-2, Eq. 24-25) on the GPU with the
library's own kernels.

Data: mean patches of noisy/clean groups (the pairs Sec. III-E-2 says overlapping groups supply
in abundance).  Seeded clean synthetic images (half of them with the 1/f texture) and 512 x 512
crops of large textured ones (1536 x 2048, whose shapes are as large as those of multi-megapixel
images) get Gaussian noise of sigma U[30, 75] (the range where the enhancement applies, Sec.
IV-B); the groups are
matched on the noisy image (htsvd_block_match, K 16 and 32), and htsvd_ra_means averages them
over the noisy and over the clean image.  Training minimises the mean of
(r - (noisy - clean)/128)^2 with htsvd_ra_train_step (forward, backward and Adam in HIP);
PyTorch only holds the device buffers.

    python -m paper_2512_23569_amd.train_ra --c 3 --images 600 --big 120 --epochs 16
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

TRAIN_SEED0 = 50000     # image seeds of the training set
HOLDOUT_SEED0 = 60000   # and of the held-out set


def init_params(c: int, seed: int) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)) and zero biases, in the flattened order
    W1, b1, W2, b2, W3, b3 of the library's network."""
    P, H = 64 * c, (256 if c == 3 else 128)
    rng = np.random.default_rng(seed)
    parts = []
    for rows, cols in ((H, P), (H, H), (P, H)):
        b = np.sqrt(6.0 / cols)
        parts += [rng.uniform(-b, b, rows * cols), np.zeros(rows)]
    return np.concatenate(parts).astype(np.float32)


def _pair(args):
    seed, size, c = args
    rng = np.random.default_rng(seed)
    sigma = float(rng.uniform(30.0, 75.0))
    clean = synth.make_clean(size, size, c, seed, texture=bool(seed % 2))
    noisy = synth.add_awgn(clean, sigma, seed + 7)
    return clean, noisy, sigma


def _pair_big(args):
    seed, size, c = args
    rng = np.random.default_rng(seed)
    sigma = float(rng.uniform(30.0, 75.0))
    full = synth.make_clean(1536, 2048, c, seed, texture=True)
    y, x = int(rng.integers(0, 1536 - size + 1)), int(rng.integers(0, 2048 - size + 1))
    clean = np.ascontiguousarray(full[y:y + size, x:x + size])
    noisy = synth.add_awgn(clean, sigma, seed + 7)
    return clean, noisy, sigma


def make_images(first_seed, n, size, c, workers=8, big=False):
    if n <= 0:
        return []
    jobs = [(first_seed + i, size, c) for i in range(n)]
    with Pool(workers) as pool:
        return pool.map(_pair_big if big else _pair, jobs, chunksize=1 if big else 4)


def mean_pairs(ht, dn, images, c, Ks=(16, 32)):
    """Noisy and clean mean patches of every group of every image, on the device."""
    import torch
    noisy_m, clean_m = [], []
    for clean, noisy, _ in images:
        dc = torch.from_numpy(np.ascontiguousarray(clean)).cuda()
        dnz = torch.from_numpy(np.ascontiguousarray(noisy)).cuda()
        for K in Ks:
            p = dn.params(c, stride=4, window=31 if c == 3 else 21, K=K)
            idx, _ = dn.block_match(dnz, p, with_dist=False)
            noisy_m.append(dn.ra_means(dnz, idx, K))
            clean_m.append(dn.ra_means(dc, idx, K))
    return torch.cat(noisy_m), torch.cat(clean_m)


def evaluate(ht, ctx, c, xn, xc, batch, grad):
    tot, n = 0.0, xn.shape[0]
    for i in range(0, n, batch):
        b = min(batch, n - i)
        tot += ht.htsvd_ra_gradients(ctx, c, xn[i:i + b], xc[i:i + b], b, grad) * b
    return tot / n


def psnr_gain(ht, dn, images, c, K=32):
    """Mean PSNR of the denoiser with and without the refinement on held-out images (known sigma)."""
    import torch
    with_ra, without = [], []
    for clean, noisy, sigma in images:
        d = torch.from_numpy(np.ascontiguousarray(noisy)).cuda()
        p = dn.params(c, stride=4, window=31 if c == 3 else 21, K=K)
        a = dn.denoise(d, sigma, p).cpu().numpy()
        b = dn.denoise(d, sigma, p.replace(ra=1)).cpu().numpy()
        without.append(synth.psnr(clean, a))
        with_ra.append(synth.psnr(clean, b))
    return float(np.mean(with_ra)), float(np.mean(without))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--c", type=int, default=3)
    ap.add_argument("--images", type=int, default=240)
    ap.add_argument("--holdout", type=int, default=16)
    ap.add_argument("--big", type=int, default=0, help="512 x 512 crops of large textured images added")
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", type=str, default=None)
    args = ap.parse_args(argv)
    import torch

    import paper_2512_23569_amd as ht
    c = args.c
    out = args.out or os.path.join(ht.DATA_DIR, "ra_fcn_c%d.f32" % c)
    t0 = time.time()
    train_imgs = make_images(TRAIN_SEED0, args.images, args.size, c)
    train_imgs += make_images(TRAIN_SEED0 + 5000, args.big, 512, c, big=True)
    hold_imgs = make_images(HOLDOUT_SEED0, args.holdout, args.size, c)
    hold_big = make_images(HOLDOUT_SEED0 + 5000, 6, 512, c, big=True)
    print("images in %.1f s" % (time.time() - t0), flush=True)
    dn = ht.Denoiser(0, load_network=False)
    ht.htsvd_ra_set_weights(dn.ctx, c, init_params(c, args.seed))
    xn, xc = mean_pairs(ht, dn, train_imgs, c)
    hn, hc = mean_pairs(ht, dn, hold_imgs, c)
    n = xn.shape[0]
    print("pairs: %d training, %d held out (%.1f s)" % (n, hn.shape[0], time.time() - t0), flush=True)
    grad = torch.empty(ht.htsvd_ra_param_count(c), dtype=torch.float32, device="cuda")
    log = {"c": c, "images": args.images, "size": args.size, "pairs": n, "epochs": args.epochs, "batch": args.batch,
           "lr": args.lr, "holdout_loss": [evaluate(ht, dn.ctx, c, hn, hc, args.batch, grad)]}
    gen = torch.Generator(device="cuda")
    gen.manual_seed(args.seed)
    steps = 0
    for ep in range(args.epochs):
        lr = args.lr * (0.5 ** max(0, ep - args.epochs // 2))
        perm = torch.randperm(n, device="cuda", generator=gen)
        tot = 0.0
        for i in range(0, n - args.batch + 1, args.batch):
            sel = perm[i:i + args.batch]
            loss = ht.htsvd_ra_train_step(dn.ctx, c, xn[sel].contiguous(), xc[sel].contiguous(), args.batch, lr)
            tot += loss
            steps += 1
        hl = evaluate(ht, dn.ctx, c, hn, hc, args.batch, grad)
        log["holdout_loss"].append(hl)
        print("epoch %d: lr %.2g, train %.6f, held out %.6f (%.1f s)"
              % (ep, lr, tot / max(1, n // args.batch), hl, time.time() - t0), flush=True)
    w = ht.htsvd_ra_get_weights(dn.ctx, c)
    w.astype("<f4").tofile(out)
    gain = psnr_gain(ht, dn, hold_imgs, c)
    gain_big = psnr_gain(ht, dn, hold_big, c)
    log.update({"big": args.big, "steps": steps, "holdout_psnr_ra": gain[0], "holdout_psnr_plain": gain[1],
                "holdout_big_psnr_ra": gain_big[0], "holdout_big_psnr_plain": gain_big[1],
                "seconds": round(time.time() - t0, 1)})
    print("held-out PSNR with the refinement %.3f dB, without %.3f dB" % gain, flush=True)
    print("held-out large-image crops: with the refinement %.3f dB, without %.3f dB" % gain_big, flush=True)
    with open(out + ".json", "w") as f:
        json.dump(log, f, indent=1)
    dn.close()


if __name__ == "__main__":
    main()
