"""Autotuner of the batched form: the group-size policy and the launch shape.

Two decisions are made on the GPU, by measurement, and cached as JSON:

* ``k_sigma_cutoff``: the group size K trades quality for time (the transform work per group is
  linear in K).  On seeded synthetic images with known noise, the tuner denoises every noise
  level of a grid with K = 16 and K = 32 and keeps the largest level below which the PSNR lost
  by K = 16 stays within a budget.  Images whose mean estimated noise level falls below the
  cutoff then run with K = 16; the decision itself is taken on the device (HTSVD_K_AUTO).
* ``blocks_per_cu`` and ``tile_side``: the persistent grid size and the side of the filter's
  reference tiles, timed on the batch itself (graph replays, median of a few runs).

The calibration images use their own seeds, disjoint from any benchmark batch.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

CACHE_ENV = "HTSVD_TUNE_CACHE"


def _cache_path():
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache", "htsvd", "tune.json")


def _load_cache():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(d):
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path + ".tmp", "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)
    except OSError:
        pass


def device_key():
    import torch
    p = torch.cuda.get_device_properties(0)
    return "%s/%d" % (getattr(p, "gcnArchName", p.name), p.multi_processor_count)


def calibrate_k_cutoff(dn, params, sigmas=tuple(range(5, 80, 5)), shape=(384, 512), seeds=(70001, 70002),
                       budget_db=0.05):
    """Largest noise level s_c such that, for every grid level below s_c, K = 16 loses at most
    budget_db of PSNR against K = 32 (mean over the seeds).  Returns (cutoff, table)."""
    import torch

    import synth
    h, w = shape
    c = 3
    table = []
    for s in sigmas:
        loss = []
        for seed in seeds:
            clean = synth.make_clean(h, w, c, seed)
            noisy = synth.add_awgn(clean, float(s), seed + 1)
            x = torch.from_numpy(noisy).cuda()
            o16 = dn.denoise(x, float(s), params.replace(K=16)).cpu().numpy()
            o32 = dn.denoise(x, float(s), params.replace(K=32)).cpu().numpy()
            loss.append(synth.psnr(clean, o32) - synth.psnr(clean, o16))
        table.append({"sigma": float(s), "psnr_loss_k16_db": float(np.mean(loss))})
    cutoff = 0.0
    for row in table:
        if row["psnr_loss_k16_db"] > budget_db:
            break
        cutoff = row["sigma"] + 0.5 * (sigmas[1] - sigmas[0]) if len(sigmas) > 1 else row["sigma"]
    return cutoff, table


def tune_launch(dn, imgs, sigmas, params, Ks, cutoff, outs, blocks=(1, 2), sides=(16, 12, 8), reps=3):
    """Times the batch graph for each (blocks_per_cu, tile_side) and returns the fastest."""
    import torch
    results = []
    for b in blocks:
        for t in sides:
            kw = dict(Ks=Ks, outs=outs, use_graph=True, blocks_per_cu=b, k_sigma_cutoff=cutoff, tile_side=t)
            dn.denoise_batch(imgs, sigmas, params, **kw)      # capture
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                dn.denoise_batch(imgs, sigmas, params, **kw)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            results.append({"blocks_per_cu": b, "tile_side": t, "ms": 1e3 * float(np.median(ts))})
    best = min(results, key=lambda r: r["ms"])
    return best, results


def k_cutoff(dn, params, budget_db=0.05, retune=False):
    """Cached calibration of the group-size cutoff for this device and parameter set."""
    key = "kcut/%s/s%d/W%d/a%d/b%.3f" % (device_key(), params.stride, params.window, params.adaptive, budget_db)
    cache = _load_cache()
    if not retune and key in cache:
        return cache[key]["cutoff"], cache[key]["table"]
    cut, table = calibrate_k_cutoff(dn, params, budget_db=budget_db)
    cache[key] = {"cutoff": cut, "table": table}
    _store_cache(cache)
    return cut, table


def launch_shape(dn, imgs, sigmas, params, Ks, cutoff, outs, retune=False):
    """Cached launch shape for a batch signature (sizes and group sizes, not contents)."""
    sizes = sorted((int(x.shape[0]), int(x.shape[1])) for x in imgs)
    sig = hash((tuple(sizes), tuple(Ks), params.stride, params.window)) & 0xFFFFFFFF
    key = "launch/%s/%08x" % (device_key(), sig)
    cache = _load_cache()
    if not retune and key in cache:
        return cache[key]["best"], cache[key]["all"]
    best, allr = tune_launch(dn, imgs, sigmas, params, Ks, cutoff, outs)
    cache[key] = {"best": best, "all": allr}
    _store_cache(cache)
    return best, allr
