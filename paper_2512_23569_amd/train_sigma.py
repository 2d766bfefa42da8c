"""Trains the learned noise-level network on the GPU with the library's own kernels.

Data: seeded synthetic crops (synth.sigma_crop): clean synthetic images plus Gaussian noise
whose sigma varies smoothly over the crop (4x4 grid of U[5,75] values, bilinear), labelled
with log of the RMS sigma of every 8x8 block.  Training uses htsvd_cnn_train_step (forward,
backward and Adam in HIP); PyTorch only holds the device buffers.

    python -m paper_2512_23569_amd.train_sigma --crops 20000 --epochs 4 --out sigma_cnn_c3.ckpt
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402


def _crop(args):
    seed, size, c = args
    noisy, label, _ = synth.sigma_crop(seed, size, c)
    return noisy, label


def make_set(first_seed: int, n: int, size: int = 128, c: int = 3, workers: int = 8):
    jobs = [(first_seed + i, size, c) for i in range(n)]
    if workers > 1:
        with Pool(workers) as pool:
            out = pool.map(_crop, jobs, chunksize=64)
    else:
        out = [_crop(j) for j in jobs]
    x = np.stack([o[0] for o in out]).reshape(n, size, size, c)
    y = np.stack([o[1] for o in out])
    return np.ascontiguousarray(x), np.ascontiguousarray(y.astype(np.float32))


def evaluate(ht, ctx, d_x, d_y, n, size, c, batch, grad_buf):
    tot = 0.0
    for i in range(0, n, batch):
        b = min(batch, n - i)
        tot += ht.htsvd_cnn_gradients(ctx, d_x[i:i + b], b, size, size, c, d_y[i:i + b], grad_buf) * b
    return tot / n


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--crops", type=int, default=20000)
    ap.add_argument("--holdout", type=int, default=1000)
    ap.add_argument("--size", type=int, default=128)
    ap.add_argument("--c", type=int, default=3)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--init-seed", type=int, default=1)
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--out", type=str, required=True)
    ap.add_argument("--resume", type=str, default=None)
    args = ap.parse_args(argv)

    import torch

    import paper_2512_23569_amd as ht

    t0 = time.time()
    x, y = make_set(args.seed, args.crops, args.size, args.c, args.workers)
    xv, yv = make_set(10 ** 6, args.holdout, args.size, args.c, args.workers)
    print("data: %d train / %d held-out crops in %.1f s" % (args.crops, args.holdout, time.time() - t0), flush=True)

    dn = ht.Denoiser(0, load_network=False)
    ctx = dn.ctx
    if args.resume:
        ht.htsvd_cnn_load(ctx, args.resume)
    else:
        ht.htsvd_cnn_init(ctx, args.c, args.init_seed)
    dev = torch.device("cuda:0")
    d_xv = torch.from_numpy(xv).to(dev)
    d_yv = torch.from_numpy(yv).to(dev)
    grad_buf = torch.empty(ht.htsvd_cnn_param_count(args.c), dtype=torch.float32, device=dev)
    rng = np.random.Generator(np.random.PCG64(args.seed + 17))
    steps_per_epoch = args.crops // args.batch
    total = steps_per_epoch * args.epochs
    step = 0
    log = []
    v0 = evaluate(ht, ctx, d_xv, d_yv, args.holdout, args.size, args.c, 64, grad_buf)
    print("held-out |log sigma error| before: %.4f" % v0, flush=True)
    for ep in range(args.epochs):
        perm = rng.permutation(args.crops)
        d_x = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
        d_y = torch.from_numpy(np.ascontiguousarray(y[perm])).to(dev)
        te = time.time()
        run = 0.0
        for i in range(steps_per_epoch):
            lr = args.lr * 0.5 * (1.0 + math.cos(math.pi * step / total))
            sl = slice(i * args.batch, (i + 1) * args.batch)
            want = (i % 50) == 0
            loss = ht.htsvd_cnn_train_step(ctx, d_x[sl], args.batch, args.size, args.size, args.c, d_y[sl], lr,
                                           want_loss=want)
            if want:
                run = loss
            step += 1
        torch.cuda.synchronize()
        v = evaluate(ht, ctx, d_xv, d_yv, args.holdout, args.size, args.c, 64, grad_buf)
        rec = {"epoch": ep + 1, "train_loss_last": round(run, 5), "heldout_mae_log_sigma": round(v, 5),
               "epoch_s": round(time.time() - te, 2)}
        log.append(rec)
        print(json.dumps(rec), flush=True)
    ht.htsvd_cnn_save(ctx, args.out)
    print("saved %s (%d steps)" % (args.out, step), flush=True)
    dn.close()
    return log


if __name__ == "__main__":
    main()
