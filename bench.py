"""Benchmark: Mpixel/s of Haar-tSVD denoising on one MI355X, plain form vs batched + learned form.

Workloads (seeded synthetic inputs, uint8, resident in HBM before the timed region):

* 12 MP: one 4000x3000 RGB image (generator with 1/f texture), AWGN sigma = 50; ps 8,
  reference stride 3, search window 31.  The noise level is not given to the method: it is
  estimated (adaptive mode, sub-images of 128).
    - plain form: htsvd_denoise, eigenvalue estimator + vote, K = 32.  This is ``value``.
    - batched + learned form: htsvd_denoise_batch (persistent kernels, one hipGraph replay),
      learned sigma map judged by the plain estimate, vote, group size chosen on the device
      from the autotuned sigma cutoff.
* batch: 64 RGB images, sizes uniform over {256x256, 512x384, 1024x768, 1920x1080, 2048x1536},
  AWGN sigma uniform in [5, 75]; stride 4, window 31.
    - plain form: 64 htsvd_denoise calls in sequence on one stream (plain estimator, K = 32).
    - batched + learned form: one graph replay over the whole batch.

A step is one pass of the whole path (grouping, noise level, transform, threshold, inverse,
aggregation) over the workload.  Equal quality is checked as the PSNR difference of the two
forms (mean over the batch images).

The roofline figure is for the dominant kernel, the group filter of the plain form at 12 MP
(filter_mfma_kernel<3,32>), timed live with HIP events that the library records on the stream
it launches on; its algorithmic FLOPs per group are those of the Fourier-route t-product (5120
real MACs per patch and direction for c = 3) plus the Haar butterflies, against the FP32 peak.
The FLOPs the matrix cores actually execute (fp16 hi/lo products of the per-slice maps) are
reported beside it against the fp16 matrix peak.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published FP32 vector peak, 157.3 TFLOP/s, counts packed FP32 (two values per
# instruction).  The library is built with packed FP32 switched off, so its vector code can reach
# at most half of it, 78.6 TFLOP/s; both fractions are reported.
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_FP32_UNPACKED_TFLOPS = 78.6
PEAK_INT8_MFMA_TOPS = 5000.0     # MI355X dense int8 matrix peak
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "filter_mfma_12mp_traffic.json")
FILTER_SRC = os.path.join(ROOT, "paper_2512_23569_amd", "csrc", "filter_mfma.hip")
PEAK_F16_MFMA_TFLOPS = 2500.0    # MI355X dense fp16 matrix peak
GRAM_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gram_kernel_12mp_traffic.json")
VIDEO_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "filter_mfma_ga_video_7x1080p_traffic.json")
GRAM_SRC = os.path.join(ROOT, "paper_2512_23569_amd", "csrc", "basis_learn.hip")
BAND_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "band_filter_512x512x31_traffic.json")
BAND_SRC = os.path.join(ROOT, "paper_2512_23569_amd", "csrc", "bands.hip")
RA_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fcn_fwd_12mp_traffic.json")
RA_SRC = os.path.join(ROOT, "paper_2512_23569_amd", "csrc", "ra.hip")


def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print("[bench %s] %s" % (time.strftime("%H:%M:%S"), msg), file=sys.stderr, flush=True)


def filter_flops_per_group(K: int, c: int) -> float:
    """Algorithmic FP32 FLOPs of one group: forward + inverse patch transforms and Haar."""
    per_patch_dir = (2 * 512 + 2 * 4 * 512) * 2 if c == 3 else 2 * 512 * 2
    haar = 2 * (K - 1) * 64 * c * 3  # per butterfly pair: 1 add, 1 sub, 2 mul -> 3 flop per output, 2 passes
    return 2 * K * per_patch_dir + haar


def filter_mfma_flops_per_group(K: int, c: int) -> float:
    """FLOPs the matrix cores execute per group (32x32x16 fp16 products, 32768 FLOP each):
    per 32 patches, forward 2 x (8 + 32 c=3 blocks) products, inverse 3 x as many."""
    blocks = 40 if c == 3 else 8
    return (2 + 3) * blocks * 32768.0 * (K / 32.0)


def bm_int8_ops(h: int, w: int, s: int, W: int) -> float:
    """Algorithmic int8 operations of block matching: every reference against every candidate
    of its clipped window, 64 multiply-adds (2 ops) per pair (the 8x8 patch of one plane)."""
    import oracle
    R = (W - 1) // 2

    def side(n):
        ys = oracle.ref_grid(n, 8, s)
        return sum(min(int(y) + R, n - 8) - max(int(y) - R, 0) + 1 for y in ys)
    return 2.0 * 64 * side(h) * side(w)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def source_hash(path: str) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def filter_source_hash() -> str:
    return source_hash(FILTER_SRC)


def measured_traffic(kernel_launch_refs: int, traffic_file: str = TRAFFIC_FILE, src: str = FILTER_SRC,
                     hash_key: str = "filter_src_sha256_16", size_key: str = "n_ref"):
    """HBM bytes per launch of a kernel from its committed counter summary, for the launch
    size it was measured at; None when the summary is missing, the size differs or the kernel
    source changed since."""
    try:
        with open(traffic_file) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get(hash_key) != source_hash(src) or t.get(size_key) != kernel_launch_refs:
        return None
    return t.get("bytes_per_launch")


def _gen_batch_image(spec):
    import synth
    h, w, sigma, seed = spec
    clean = synth.make_clean(h, w, 3, seed)
    return clean, synth.add_awgn(clean, sigma, seed + 1000)


def time_steps(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target duration of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-image workload")
    ap.add_argument("--plain-only", action="store_true", help="time only the plain form at 12 MP (profiling)")
    ap.add_argument("--batch-n", type=int, default=64)
    ap.add_argument("--size", type=str, default="3000x4000", help="HxW of the single image (default 12 MP)")
    ap.add_argument("--retune", action="store_true", help="ignore the autotuner cache")
    ap.add_argument("--learn-basis", action="store_true",
                    help="time the per-image learned basis instead: learn (U, V) from the noisy 12 MP image, "
                         "then denoise with it")
    ap.add_argument("--sweep", action="store_true",
                    help="time a parameter sweep instead: sigma in {30..70} x K in {16, 32} with one grouping pass, "
                         "against one call per setting")
    ap.add_argument("--ra", action="store_true",
                    help="time RA-Haar-tSVD instead: the plain form with the refinement network of the first "
                         "Haar row, against the plain form")
    ap.add_argument("--bands", action="store_true",
                    help="time the hyperspectral path instead: a 512x512x31 cube, basis learned from it, "
                         "tube patches 8x8x31")
    ap.add_argument("--video", action="store_true",
                    help="time the video path instead: 7 frames of 1080x1920 RGB, spatio-temporal grouping over "
                         "3 frames, K 32")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        a = torch.ones(args.copy_probe << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 4, "launches": 3}), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(whole images or row strips would shard across GPUs).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2512_23569_amd as ht
    import synth
    from paper_2512_23569_amd import autotune

    if args.bands:
        bench_bands(args)
        return
    if args.video:
        bench_video(args)
        return

    AUTO, KAUTO = ht.HTSVD_SIGMA_AUTO, ht.HTSVD_K_AUTO
    h, w = (int(v) for v in args.size.split("x"))
    sigma, s, W, c = 50.0, 3, 31, 3
    t0 = time.time()
    clean = synth.make_clean(h, w, 3, seed=3, texture=True)
    noisy = synth.add_awgn(clean, sigma, seed=1003)
    gen_s = time.time() - t0
    log("12 MP input generated in %.1f s" % gen_s)

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    d_in = torch.from_numpy(noisy).to(dev)
    d_out = torch.empty((h, w, c), dtype=torch.float32, device=dev)
    dn = ht.Denoiser(0)
    p_plain = dn.params(3, stride=s, window=W, K=32, adaptive=1, estimator=0)
    p_learn = p_plain.replace(estimator=1)

    if args.ra:
        bench_ra(dn, args, clean, noisy, d_in, d_out, p_plain, stream, s, W, sigma, gen_s)
        dn.close()
        return

    if args.sweep:
        bench_sweep(dn, args, clean, d_in, stream, s, W, sigma, gen_s)
        dn.close()
        return

    if args.learn_basis:
        bench_learn_basis(dn, args, clean, noisy, d_in, d_out, p_plain, stream, s, sigma, gen_s)
        dn.close()
        return

    # ---- 12 MP, plain form (value), with stage timing for the roofline ----
    plain_fn = lambda: dn.denoise(d_in, AUTO, p_plain, out=d_out)  # noqa: E731
    for _ in range(args.warmup):
        plain_fn()
    torch.cuda.synchronize()
    ht.htsvd_set_timing(dn.ctx, True)
    ms_plain = time_steps(plain_fn, args.steps, 0, stream)
    stages = ht.htsvd_stage_times(dn.ctx)
    ht.htsvd_set_timing(dn.ctx, False)
    guard = ht.htsvd_last_guard_count(dn.ctx)
    psnr_plain = synth.psnr(clean, d_out.cpu().numpy())
    psnr_in = synth.psnr(clean, noisy)
    mpx_plain = h * w / (ms_plain * 1e-3) / 1e6
    log("12 MP plain form: %.2f ms/step, %.1f Mpx/s, PSNR %.3f, guard %s" % (ms_plain, mpx_plain, psnr_plain, guard))

    ny, nx = ht.htsvd_ref_count(h, 8, s), ht.htsvd_ref_count(w, 8, s)
    n_ref = ny * nx
    fl = filter_flops_per_group(32, c) * n_ref
    f_ms, f_calls = stages["filter"]
    f_avg_ms = f_ms / max(f_calls, 1)
    achieved_tf = fl / (f_avg_ms * 1e-3) / 1e12
    mf_tf = filter_mfma_flops_per_group(32, c) * n_ref / (f_avg_ms * 1e-3) / 1e12
    traffic = measured_traffic(n_ref)
    bm_ms, bm_calls = stages["bm"]
    bm_avg_ms = bm_ms / max(bm_calls, 1)
    bm_ops = bm_int8_ops(h, w, s, W)
    alg_bytes = h * w * c * (1 + 4)      # uint8 in, float32 out

    result = {
        "metric": "Mpixel/s denoised, 12MP RGB sigma=50, plain vs batched+learned at equal PSNR",
        "value": round(mpx_plain, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_plain, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp16x2-split MFMA, f32 accumulate, f64 guard band; int8 MFMA grouping",
        "data": "synthetic",
        "config": {"workload": "12MP RGB %dx%d, AWGN sigma=%g estimated (plain estimator + vote), ps 8, stride %d, "
                               "window %d, K 32" % (w, h, sigma, s, W),
                   "form": "plain", "n_ref": n_ref},
        "roofline": {"bound": "alu", "kernel": "filter_mfma_kernel<3,32>", "achieved": round(achieved_tf, 3),
                     "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved_tf / PEAK_FP32_VECTOR_TFLOPS, 4),
                     "frac_unpacked_fp32": round(achieved_tf / PEAK_FP32_UNPACKED_TFLOPS, 4),
                     "traffic": traffic,
                     "hbm_frac": (round(traffic / (f_avg_ms * 1e-3) / (PEAK_HBM_GBS * 1e9), 5) if traffic else None),
                     "kernel_ms": round(f_avg_ms, 4), "flop_per_launch": fl,
                     "mfma": {"dtype": "f16", "executed_tflops": round(mf_tf, 3), "peak": PEAK_F16_MFMA_TFLOPS,
                              "frac": round(mf_tf / PEAK_F16_MFMA_TFLOPS, 4)}},
        "hbm_algorithmic": {"bytes_per_step": alg_bytes, "gbs": round(alg_bytes / (ms_plain * 1e-3) / 1e9, 2),
                            "frac": round(alg_bytes / (ms_plain * 1e-3) / (PEAK_HBM_GBS * 1e9), 5)},
        "block_matching": {"kernel": "bm_kernel", "int8_ops": bm_ops, "ms": round(bm_avg_ms, 4),
                           "tops": round(bm_ops / (bm_avg_ms * 1e-3) / 1e12, 2),
                           "int8_mfma_frac": round(bm_ops / (bm_avg_ms * 1e-3) / 1e12 / PEAK_INT8_MFMA_TOPS, 5)},
        "guard": {"fp64_redecided": int(guard[0]), "fp32_beyond_list": int(guard[1])},
        "stages_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in stages.items() if v[1]},
        "psnr": {"noisy": round(psnr_in, 3), "plain": round(psnr_plain, 3)},
        "input_gen_s": round(gen_s, 1),
    }

    if not args.plain_only:
        # ---- autotuner: group-size cutoff (calibrated on its own seeds) ----
        t0 = time.time()
        cutoff, table = autotune.k_cutoff(dn, p_plain, retune=args.retune)
        log("k cutoff %.1f (%.1f s)" % (cutoff, time.time() - t0))
        result["autotune"] = {"k_sigma_cutoff": cutoff, "calib_s": round(time.time() - t0, 1),
                              "psnr_loss_k16_db": {int(r["sigma"]): round(r["psnr_loss_k16_db"], 3) for r in table}}

        # ---- 12 MP, plain form at K = 16 (the group size the autotuner picks) ----
        p_plain16 = p_plain.replace(K=16)
        ms_p16 = time_steps(lambda: dn.denoise(d_in, AUTO, p_plain16, out=d_out), args.steps, args.warmup, stream)
        psnr_p16 = synth.psnr(clean, d_out.cpu().numpy())
        log("12 MP plain form K 16: %.2f ms/step, PSNR %.3f" % (ms_p16, psnr_p16))
        result["plain_k16_12mp"] = {"value": round(h * w / (ms_p16 * 1e-3) / 1e6, 3), "ms_per_step": round(ms_p16, 3),
                                    "psnr": round(psnr_p16, 3), "K": 16}

        # ---- 12 MP, batched + learned form ----
        bl_kw = dict(Ks=[KAUTO], outs=[d_out], use_graph=True, k_sigma_cutoff=cutoff)
        bl_fn = lambda: dn.denoise_batch([d_in], [AUTO], p_learn, **bl_kw)  # noqa: E731
        ms_bl = time_steps(bl_fn, args.steps, args.warmup, stream)
        psnr_bl = synth.psnr(clean, d_out.cpu().numpy())
        k_bl = ht.htsvd_batch_inspect(dn.ctx, 0)
        log("12 MP batched+learned form: %.2f ms/step, PSNR %.3f, K %d" % (ms_bl, psnr_bl, k_bl))
        result["batched_learned_12mp"] = {
            "value": round(h * w / (ms_bl * 1e-3) / 1e6, 3), "ms_per_step": round(ms_bl, 3),
            "psnr": round(psnr_bl, 3), "K": k_bl, "speedup_vs_plain": round(ms_plain / ms_bl, 3),
            "dpsnr_vs_plain_db": round(psnr_bl - psnr_plain, 3),
            "speedup_same_k": round(ms_p16 / ms_bl, 3) if k_bl == 16 else None,
            "dpsnr_vs_plain_same_k_db": round(psnr_bl - psnr_p16, 3) if k_bl == 16 else None}

    if not args.no_batch and not args.plain_only:
        result["batch"] = bench_batch(dn, args, autotune, stream)

    if not args.no_cpu_baseline and not args.plain_only:
        result["cpu_baseline"] = cpu_baseline(noisy, s, W, 32, sigma, args.cpu_seconds)

    print(json.dumps(result), flush=True)
    dn.close()


def bench_batch(dn, args, autotune, stream):
    """The 64-image workload: plain per-image calls vs one batched + learned graph replay."""
    from multiprocessing import Pool

    import numpy as np
    import torch

    import paper_2512_23569_amd as ht
    import synth
    AUTO, KAUTO = ht.HTSVD_SIGMA_AUTO, ht.HTSVD_K_AUTO
    specs = synth.batch_specs(args.batch_n, seed=4)
    t0 = time.time()
    with Pool(min(16, os.cpu_count() or 1)) as pool:
        pairs = pool.map(_gen_batch_image, specs)
    gen_s = time.time() - t0
    log("batch of %d generated in %.1f s" % (len(pairs), gen_s))
    ins = [torch.from_numpy(nz).cuda() for _, nz in pairs]
    outs = [torch.empty(x.shape, dtype=torch.float32, device="cuda") for x in ins]
    total_px = sum(x.shape[0] * x.shape[1] for x in ins)
    p_plain = dn.params(3, stride=4, window=31, K=32, adaptive=1, estimator=0)
    p_learn = p_plain.replace(estimator=1)
    cutoff, _ = autotune.k_cutoff(dn, p_plain, retune=args.retune)

    def plain():
        for x, o in zip(ins, outs):
            dn.denoise(x, AUTO, p_plain, out=o)

    ms_plain = time_steps(plain, args.steps, args.warmup, stream)
    psnr_plain = [synth.psnr(cl, o.cpu().numpy()) for (cl, _), o in zip(pairs, outs)]
    log("batch plain form: %.2f ms/step, mean PSNR %.3f" % (ms_plain, float(np.mean(psnr_plain))))
    p_plain16 = p_plain.replace(K=16)

    def plain16():
        for x, o in zip(ins, outs):
            dn.denoise(x, AUTO, p_plain16, out=o)

    ms_p16 = time_steps(plain16, args.steps, args.warmup, stream)
    psnr_p16 = [synth.psnr(cl, o.cpu().numpy()) for (cl, _), o in zip(pairs, outs)]
    log("batch plain form K 16: %.2f ms/step, mean PSNR %.3f" % (ms_p16, float(np.mean(psnr_p16))))

    Ks = [KAUTO] * len(ins)
    sig = [AUTO] * len(ins)
    t0 = time.time()
    best, allr = autotune.launch_shape(dn, ins, sig, p_learn, Ks, cutoff, outs, retune=args.retune)
    tune_s = time.time() - t0
    log("batch launch shape %s (%.1f s)" % (best, tune_s))
    kw = dict(Ks=Ks, outs=outs, use_graph=True, k_sigma_cutoff=cutoff, blocks_per_cu=best["blocks_per_cu"],
              tile_side=best["tile_side"])
    ms_bl = time_steps(lambda: dn.denoise_batch(ins, sig, p_learn, **kw), args.steps, args.warmup, stream)
    psnr_bl = [synth.psnr(cl, o.cpu().numpy()) for (cl, _), o in zip(pairs, outs)]
    k_used = [ht.htsvd_batch_inspect(dn.ctx, i) for i in range(len(ins))]
    dps = float(np.mean(psnr_bl) - np.mean(psnr_plain))
    dps16 = float(np.mean(psnr_bl) - np.mean(psnr_p16))
    log("batch batched+learned form: %.2f ms/step, mean PSNR %.3f" % (ms_bl, float(np.mean(psnr_bl))))
    return {
        "workload": "%d RGB images (%.1f MP total), AWGN sigma U[5,75] estimated, stride 4, window 31"
                    % (len(ins), total_px / 1e6),
        "plain": {"value": round(total_px / (ms_plain * 1e-3) / 1e6, 3), "ms_per_step": round(ms_plain, 3),
                  "mean_psnr": round(float(np.mean(psnr_plain)), 3), "K": 32},
        "plain_k16": {"value": round(total_px / (ms_p16 * 1e-3) / 1e6, 3), "ms_per_step": round(ms_p16, 3),
                      "mean_psnr": round(float(np.mean(psnr_p16)), 3), "K": 16},
        "batched_learned": {"value": round(total_px / (ms_bl * 1e-3) / 1e6, 3), "ms_per_step": round(ms_bl, 3),
                            "mean_psnr": round(float(np.mean(psnr_bl)), 3), "launch": best,
                            "k_sigma_cutoff": cutoff, "images_at_k16": int(sum(k == 16 for k in k_used)),
                            "images_at_k32": int(sum(k == 32 for k in k_used))},
        "speedup": round(ms_plain / ms_bl, 3),
        "dpsnr_db": round(dps, 3),
        "psnr_within_0p05_db": bool(abs(dps) <= 0.05),
        "psnr_not_worse_than_0p05_db": bool(dps >= -0.05),
        "speedup_same_k": round(ms_p16 / ms_bl, 3),
        "dpsnr_same_k_db": round(dps16, 3),
        "psnr_within_0p05_db_same_k": bool(abs(dps16) <= 0.05),
        "unit": "Mpixel/s",
        "gen_s": round(gen_s, 1), "tune_s": round(tune_s, 1), "launch_candidates": allr,
    }


def bench_ra(dn, args, clean, noisy, d_in, d_out, p_plain, stream, s, W, sigma, gen_s):
    """RA-Haar-tSVD (Sec. III-E-2): the plain form (sigma estimated, vote) with the refinement
    network applied to every group whose noise level exceeds 30, against the plain form.  The
    roofline figure is the network kernel's, timed on the same number of mean patches through
    htsvd_ra_forward (the in-denoiser launch also averages the groups)."""
    import torch

    import paper_2512_23569_amd as ht
    import synth
    h, w, c = d_in.shape
    AUTO = ht.HTSVD_SIGMA_AUTO
    p_ra = p_plain.replace(ra=1)
    ms_plain = time_steps(lambda: dn.denoise(d_in, AUTO, p_plain, out=d_out), args.steps, args.warmup, stream)
    psnr_plain = synth.psnr(clean, d_out.cpu().numpy())
    ms_ra = time_steps(lambda: dn.denoise(d_in, AUTO, p_ra, out=d_out), args.steps, args.warmup, stream)
    psnr_ra = synth.psnr(clean, d_out.cpu().numpy())
    ny, nx = ht.htsvd_ref_count(h, 8, s), ht.htsvd_ref_count(w, 8, s)
    n_ref = ny * nx
    P, H = 64 * c, (256 if c == 3 else 128)
    means = torch.rand((n_ref, P), device=d_in.device) * 255.0
    r = torch.empty_like(means)
    ms_net = time_steps(lambda: ht.htsvd_ra_forward(dn.ctx, c, means, n_ref, r), args.steps, args.warmup, stream)
    macs = n_ref * (P * H + H * H + H * P)
    alg_tf = 2 * macs / (ms_net * 1e-3) / 1e12
    exe_tf = 3 * alg_tf   # three fp16 products per FP32 product (hi.hi, hi.lo, lo.hi)
    log("RA: %.2f ms (plain %.2f ms), PSNR %.3f (plain %.3f), network %.3f ms for %d groups"
        % (ms_ra, ms_plain, psnr_ra, psnr_plain, ms_net, n_ref))
    result = {
        "metric": "Mpixel/s denoised with RA-Haar-tSVD (refined first Haar row), 12MP RGB sigma=50",
        "value": round(h * w / (ms_ra * 1e-3) / 1e6, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_ra, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "12MP RGB %dx%d, AWGN sigma=%g estimated (plain estimator + vote), RA network on groups "
                               "with sigma > 30, ps 8, stride %d, window %d, K 32" % (w, h, sigma, s, W),
                   "form": "plain + RA", "n_ref": n_ref},
        "plain_ms": round(ms_plain, 3),
        "roofline": {"bound": "mfma", "kernel": "fcn_fwd_kernel<3>", "achieved": round(exe_tf, 3),
                     "peak": PEAK_F16_MFMA_TFLOPS, "unit": "TFLOP/s", "frac": round(exe_tf / PEAK_F16_MFMA_TFLOPS, 4),
                     "traffic": measured_traffic(n_ref, RA_TRAFFIC_FILE, RA_SRC, "src_sha256_16", "n_ref"),
                     "kernel_ms": round(ms_net, 4), "algorithmic_fp32_tflops": round(alg_tf, 3),
                     "macs_per_launch": macs},
        "psnr": {"noisy": round(synth.psnr(clean, noisy), 3), "plain": round(psnr_plain, 3), "ra": round(psnr_ra, 3)},
        "input_gen_s": round(gen_s, 1),
    }
    print(json.dumps(result), flush=True)


def bench_sweep(dn, args, clean, d_in, stream, s, W, sigma, gen_s):
    """Parameter selection (Sec. III-D-3): the same image denoised under 10 (sigma, K) settings,
    once with one grouping pass for all (htsvd_denoise_sweep, groups of 32 whose first 16
    members are the 16-member groups), once as 10 separate htsvd_denoise calls.  Reports the
    sweep's throughput in output pixels per second, the speedup, and the setting with the best
    PSNR (the selection the sweep serves)."""
    import torch

    import paper_2512_23569_amd as ht
    import synth
    h, w, c = d_in.shape
    settings = [(sg, K) for K in (16, 32) for sg in (30.0, 40.0, 50.0, 60.0, 70.0)]
    p = dn.params(3, stride=s, window=W, K=32)
    outs = [torch.empty((h, w, c), dtype=torch.float32, device=d_in.device) for _ in settings]
    sweep_fn = lambda: dn.denoise_sweep(d_in, settings, p, outs=outs)  # noqa: E731

    def singles():
        for (sg, K), o in zip(settings, outs):
            dn.denoise(d_in, sg, p.replace(K=K), out=o)

    ht.htsvd_set_timing(dn.ctx, True)
    ms_sweep = time_steps(sweep_fn, args.steps, args.warmup, stream)
    stages = ht.htsvd_stage_times(dn.ctx)
    ht.htsvd_set_timing(dn.ctx, False)
    psnrs = {"sigma%g_K%d" % st: round(synth.psnr(clean, o.cpu().numpy()), 3) for st, o in zip(settings, outs)}
    ms_single = time_steps(singles, args.steps, args.warmup, stream)
    best = max(psnrs, key=psnrs.get)
    n_out = len(settings) * h * w
    # roofline of the filter launches: mean algorithmic FLOPs of a launch over the settings
    n_ref = ht.htsvd_ref_count(h, 8, s) * ht.htsvd_ref_count(w, 8, s)
    f_ms, f_calls = stages["filter"]
    f_avg = f_ms / max(f_calls, 1)
    flop_launch = sum(filter_flops_per_group(K, c) for _, K in settings) * n_ref / len(settings)
    tf = flop_launch / (f_avg * 1e-3) / 1e12
    log("sweep of %d settings: %.2f ms (one call each: %.2f ms), best %s %.3f dB"
        % (len(settings), ms_sweep, ms_single, best, psnrs[best]))
    result = {
        "metric": "output Mpixel/s of a 10-setting parameter sweep with one grouping pass, 12MP RGB",
        "value": round(n_out / (ms_sweep * 1e-3) / 1e6, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_sweep, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "12MP RGB %dx%d, AWGN sigma=%g, known-sigma settings sigma in {30,40,50,60,70} x K in "
                               "{16,32}, ps 8, stride %d, window %d, grouping at K 32" % (w, h, sigma, s, W),
                   "form": "sweep"},
        "single_calls_ms": round(ms_single, 3),
        "speedup_vs_single_calls": round(ms_single / ms_sweep, 3),
        "stages_ms_per_launch": {k: round(v[0] / max(v[1], 1), 4) for k, v in stages.items() if v[1]},
        "roofline": {"bound": "alu", "kernel": "filter_mfma_kernel<3,16> and <3,32> (five settings each)",
                     "achieved": round(tf, 3), "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tf / PEAK_FP32_VECTOR_TFLOPS, 4),
                     "frac_unpacked_fp32": round(tf / PEAK_FP32_UNPACKED_TFLOPS, 4), "traffic": None,
                     "kernel_ms": round(f_avg, 4), "flop_per_launch": flop_launch},
        "psnr": psnrs,
        "best_setting": best,
        "input_gen_s": round(gen_s, 1),
    }
    print(json.dumps(result), flush=True)


PEAK_FP64_MFMA_TFLOPS = 78.6      # dense FP64 matrix-core peak of the MI355X


def band_flops_per_patch(B: int) -> float:
    """FP64 FLOPs of the band t-product of one patch, forward and inverse: per direction the
    band DFT and its inverse (64 x B x B real products each) and per frequency the two 8 x 8 x 8
    slice products (complex: 4 real multiply-adds per complex one; real for f = 0 and f = B/2)."""
    nf = B // 2 + 1
    n_real = 1 + (1 if B % 2 == 0 else 0)
    maps = 2 * 2 * 512 * (n_real + 4 * (nf - n_real))
    dft = 2 * 2 * 64 * B * B
    return 2.0 * (maps + dft)


def band_mfma_flops_per_patch(B: int) -> float:
    """FP64 FLOPs the matrix cores execute per patch (both directions): the band DFTs padded to
    32 or 64 bands and every slice product as four 16 x 16 x 4 steps per patch (real 16 x 16
    embeddings of the complex 8 x 8 matrices, also for the real slices)."""
    nb = 32 if B <= 32 else 64
    dft = 2 * 2 * 64 * nb * nb
    maps = (B // 2 + 1) * 4 * (2 * 16 * 16 * 4)
    return 2.0 * (dft + maps)


def bench_bands(args):
    """Hyperspectral tube patches (Sec. IV-D): a 512 x 512 x 31 cube (the size of common
    hyperspectral benchmarks), AWGN sigma 30; a step learns the basis from the noisy cube
    (Sec. III-B) and denoises it (grouping on the band-mean guide, K 16, stride 4, window 21).
    The roofline figure is the band filter's FP64 products against the FP64 vector peak."""
    import torch

    import paper_2512_23569_amd as ht
    import synth
    h, w, B, sigma = 512, 512, 31, 30.0
    t0 = time.time()
    clean = synth.make_hsi(h, w, B, seed=7)
    noisy = synth.add_awgn(clean, sigma, seed=8)
    gen_s = time.time() - t0
    stream = torch.cuda.current_stream()
    d_in = torch.from_numpy(noisy).cuda()
    d_out = torch.empty((h, w, B), dtype=torch.float32, device="cuda")
    dn = ht.Denoiser(0, load_network=False)
    p = dn.params(1, stride=4, window=21, K=16)

    def step():
        dn.learn_basis(d_in, stride=4)
        dn.denoise_bands(d_in, sigma, p, out=d_out)

    ms_step = time_steps(step, args.steps, args.warmup, stream)
    ht.htsvd_set_timing(dn.ctx, True)
    ms_den = time_steps(lambda: dn.denoise_bands(d_in, sigma, p, out=d_out), args.steps, 0, stream)
    stages = ht.htsvd_stage_times(dn.ctx)
    ht.htsvd_set_timing(dn.ctx, False)
    psnr = synth.psnr(clean, d_out.cpu().numpy())
    ny, nx = ht.htsvd_ref_count(h, 8, 4), ht.htsvd_ref_count(w, 8, 4)
    n_patch = ny * nx * 16
    # band-wise noise levels (Sec. IV-D): the same cube with non-uniform noise (levels 10..20,
    # three bands at 60), sigma AUTO, against the known mean level alone
    import numpy as np
    levels = np.linspace(10.0, 20.0, B)
    levels[[5, 17, 28]] = 60.0
    noisy_nu = synth.add_band_awgn(clean, levels, seed=9)
    d_nu = torch.from_numpy(noisy_nu).cuda()
    dn.learn_basis(d_nu, stride=4)
    ms_auto = time_steps(lambda: dn.denoise_bands(d_nu, ht.HTSVD_SIGMA_AUTO, p, out=d_out), args.steps, 1, stream)
    psnr_auto = synth.psnr(clean, d_out.cpu().numpy())
    band_sig = dn.band_sigma(d_nu)
    dn.denoise_bands(d_nu, float(np.mean(levels)), p, out=d_out)
    psnr_mean_only = synth.psnr(clean, d_out.cpu().numpy())
    log("bands, band-wise sigma: %.2f ms, PSNR %.3f (mean level only %.3f, noisy %.3f)"
        % (ms_auto, psnr_auto, psnr_mean_only, synth.psnr(clean, noisy_nu)))
    f_ms, f_calls = stages["filter"]
    f_avg = f_ms / max(f_calls, 1)
    tf = band_flops_per_patch(B) * n_patch / (f_avg * 1e-3) / 1e12
    log("bands: step %.2f ms (denoise %.2f ms, filter %.2f ms), PSNR %.3f (noisy %.3f)"
        % (ms_step, ms_den, f_avg, psnr, synth.psnr(clean, noisy)))
    result = {
        "metric": "Mpixel/s of hyperspectral denoising with a basis learned from the cube, 512x512x31, sigma=30",
        "value": round(h * w / (ms_step * 1e-3) / 1e6, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "hyperspectral cube %dx%dx%d (4 smooth endmember spectra), AWGN sigma=%g known, "
                               "tube patches 8x8x%d, grouping on the band-mean guide, stride 4, window 21, K 16"
                               % (w, h, B, sigma, B), "form": "bands"},
        "denoise_ms": round(ms_den, 3),
        "stages_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in stages.items() if v[1]},
        "roofline": {"bound": "mfma", "kernel": "band filter stage (band_tproduct_kernel<32> forward and inverse, "
                                                "haar_threshold_kernel<16>; FP64 matrix cores)", "achieved": round(tf, 3),
                     "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s", "frac": round(tf / PEAK_FP64_MFMA_TFLOPS, 4),
                     "traffic": measured_traffic(n_patch, BAND_TRAFFIC_FILE, BAND_SRC, "src_sha256_16", "n_patch"),
                     "kernel_ms": round(f_avg, 4), "flop_per_launch": band_flops_per_patch(B) * n_patch,
                     "mfma_executed_tflops": round(band_mfma_flops_per_patch(B) * n_patch / (f_avg * 1e-3) / 1e12, 3)},
        "psnr": {"noisy": round(synth.psnr(clean, noisy), 3), "denoised": round(psnr, 3)},
        "band_wise_sigma": {"levels": "10..20, bands 5, 17, 28 at 60", "ms": round(ms_auto, 3),
                            "estimated_severe": [int(b) for b in np.nonzero(band_sig > 2 * band_sig.mean())[0]],
                            "psnr": {"noisy": round(synth.psnr(clean, noisy_nu), 3), "auto": round(psnr_auto, 3),
                                     "known_mean_level_only": round(psnr_mean_only, 3)}},
        "input_gen_s": round(gen_s, 1),
    }
    if not args.no_cpu_baseline:
        import oracle
        from oracle import learn_basis as lb
        band = noisy[:64]
        t0 = time.time()
        U, V = lb.learn(band, 8, 4)
        idx, _ = oracle.block_match(oracle.band_guide(band), 8, 4, 21, 16)
        oracle.filter_groups(band, idx, U, V, sigma * np.sqrt(2.0 * np.log(B * 16 * 64)))
        dt = time.time() - t0
        cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        result["cpu_baseline"] = {"value": round(band.shape[0] * w / dt / 1e6, 5), "unit": "Mpixel/s", "cores": cores,
                                  "kind": "oracle", "sample": "the top 64 rows of the cube (%.1f s): learning, "
                                                              "grouping and filtering" % dt}
    print(json.dumps(result), flush=True)
    dn.close()


def bench_video(args):
    """Video (Sec. IV-C): 7 frames of 1080 x 1920 RGB (the frame size of common colour-video
    denoising sets) of a panning scene with a moving object, AWGN sigma 30; a step groups over
    space and time (temporal radius 1: three frames, window 15, stride 4, K 32) and filters the
    groups with the global basis on the matrix cores (global aggregation).  The roofline figure is
    the filter stage's algorithmic FP32 work against the FP32 vector peak, as for images."""
    import torch

    import paper_2512_23569_amd as ht
    import synth
    T, h, w, c, sigma, radius, K, W, s = 7, 1080, 1920, 3, 30.0, 1, 32, 15, 4
    t0 = time.time()
    clean = synth.make_video(T, h, w, c, seed=21)
    noisy = synth.add_awgn(clean, sigma, seed=22)
    gen_s = time.time() - t0
    log("video input generated in %.1f s" % gen_s)
    stream = torch.cuda.current_stream()
    d_in = torch.from_numpy(noisy).cuda()
    d_out = torch.empty(noisy.shape, dtype=torch.float32, device="cuda")
    dn = ht.Denoiser(0)   # shipped bases and networks (the RA variant below uses them)
    p = dn.params(c, stride=s, window=W, K=K)

    def step():
        dn.denoise_video(d_in, sigma, p, radius, out=d_out)

    ht.htsvd_set_timing(dn.ctx, True)
    ms_step = time_steps(step, args.steps, args.warmup, stream)
    stages = ht.htsvd_stage_times(dn.ctx)
    ht.htsvd_set_timing(dn.ctx, False)
    out = d_out.cpu().numpy()
    psnr = synth.psnr(clean, out)
    per_frame = [synth.psnr(clean[t], out[t]) for t in range(T)]
    # the other video forms on the same clip: sigma estimated frame by frame with the vote, and
    # RA-Haar-tSVD on the spatio-temporal groups (known sigma)
    variants = {}
    for name, sg, pv in (("estimated_sigma_vote", ht.HTSVD_SIGMA_AUTO, p.replace(adaptive=1)),
                         ("ra", sigma, p.replace(ra=1, ra_sigma=25.0))):
        ms_v = time_steps(lambda: dn.denoise_video(d_in, sg, pv, radius, out=d_out), max(1, args.steps // 2), 1,
                          stream)
        variants[name] = {"ms": round(ms_v, 3), "psnr": round(synth.psnr(clean, d_out.cpu().numpy()), 3)}
    log("video variants: %s" % variants)
    n_ref = T * ht.htsvd_ref_count(h, 8, s) * ht.htsvd_ref_count(w, 8, s)
    f_ms, f_calls = stages["filter"]
    f_avg = f_ms / max(f_calls, 1)
    b_ms, b_calls = stages["bm"]
    fl = filter_flops_per_group(K, c) * n_ref
    tf = fl / (f_avg * 1e-3) / 1e12
    mf_tf = filter_mfma_flops_per_group(K, c) * n_ref / (f_avg * 1e-3) / 1e12
    log("video: step %.2f ms (grouping %.2f ms, filter %.2f ms), PSNR %.3f (noisy %.3f)"
        % (ms_step, b_ms / max(b_calls, 1), f_avg, psnr, synth.psnr(clean, noisy)))
    result = {
        "metric": "Mpixel/s of video denoising, 7 frames of 1080x1920 RGB, sigma=30",
        "value": round(T * h * w / (ms_step * 1e-3) / 1e6, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "video of %d frames %dx%dx%d (panning textured scene, moving object), AWGN sigma=%g "
                               "known, spatio-temporal grouping over %d frames, stride %d, window %d, K %d"
                               % (T, w, h, c, sigma, 2 * radius + 1, s, W, K), "form": "video"},
        "stages_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in stages.items() if v[1]},
        "roofline": {"bound": "alu", "kernel": "filter_mfma_ga_kernel<3,32,false,2> + ga_gather_kernel<3> (filter stage)",
                     "achieved": round(tf, 3), "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tf / PEAK_FP32_VECTOR_TFLOPS, 4),
                     "traffic": measured_traffic(n_ref, VIDEO_TRAFFIC_FILE), "kernel_ms": round(f_avg, 4),
                     "flop_per_launch": fl,
                     "mfma": {"dtype": "f16", "executed_tflops": round(mf_tf, 3), "peak": PEAK_F16_MFMA_TFLOPS,
                              "frac": round(mf_tf / PEAK_F16_MFMA_TFLOPS, 4)}},
        "psnr": {"noisy": round(synth.psnr(clean, noisy), 3), "denoised": round(psnr, 3),
                 "per_frame": [round(v, 3) for v in per_frame]},
        "variants": variants,
        "input_gen_s": round(gen_s, 1),
    }
    if not args.no_cpu_baseline:
        import numpy as np

        import oracle
        U, V = oracle.load_basis(os.path.join(ROOT, "paper_2512_23569_amd", "data", "basis_ps8_c3.f64"), 8, 3)
        rows = h   # three whole frames
        sample = np.ascontiguousarray(noisy[:3, :rows])
        t0 = time.time()
        idx, _ = oracle.block_match_video(sample, 8, s, W, K, radius)
        oracle.filter_groups(sample.reshape(3 * rows, w, c), idx, U, V, sigma * oracle.tau_multiplier(c, K))
        dt = time.time() - t0
        cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        result["cpu_baseline"] = {"value": round(3 * rows * w / dt / 1e6, 5), "unit": "Mpixel/s", "cores": cores,
                                  "kind": "oracle", "sample": "the first 3 frames, %d rows each (%.1f s): "
                                                              "spatio-temporal grouping and filtering" % (rows, dt)}
    print(json.dumps(result), flush=True)
    dn.close()


PEAK_INT32_VALU_TOPS = 78.6   # 256 CUs x 64 lanes x 2.4 GHz x 2 (a 32-bit multiply-add counts as two ops)


def gram_ops(h, w, c, s):
    """Algorithmic integer ops of the Gram sums: every 8c-vector of the two regroupings (one per
    reference row and image column, one per reference column and image row) contributes its
    8c(8c+1)/2 distinct products, a multiply and an add each."""
    import paper_2512_23569_amd as ht
    ny, nx = ht.htsvd_ref_count(h, 8, s), ht.htsvd_ref_count(w, 8, s)
    n_vec = ny * w + nx * h
    a = 8 * c
    return n_vec, n_vec * a * (a + 1)


def bench_learn_basis(dn, args, clean, noisy, d_in, d_out, p_plain, stream, s, sigma, gen_s):
    """Per-image learned basis (Sec. III-B): a step learns (U, V) from the noisy input itself
    (Gram sums on the device, 8x8 eigendecompositions on the host, install) and denoises with it
    (plain form, sigma estimated).  The roofline figure is the Gram kernel's."""
    import numpy as np
    import torch

    import paper_2512_23569_amd as ht
    import synth
    AUTO = ht.HTSVD_SIGMA_AUTO
    h, w, c = noisy.shape
    shipped = [ht.load_basis_slices(3)]

    def step():
        dn.learn_basis(d_in, stride=s)
        dn.denoise(d_in, AUTO, p_plain, out=d_out)

    ms_step = time_steps(step, args.steps, args.warmup, stream)
    psnr_learned = synth.psnr(clean, d_out.cpu().numpy())
    # the learning call alone (host-inclusive wall time; it synchronises the stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dn.learn_basis(d_in, stride=s)
    learn_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # the Gram kernel alone (and its output clear), HIP events on the launch stream
    g = dn.basis_gram(d_in, stride=s)
    ms_gram = time_steps(lambda: ht.htsvd_basis_gram(dn.ctx, d_in, h, w, c, w * c, 8, s, g), args.steps * 5,
                         args.warmup, stream)
    # the same image denoised with the shipped basis, for the quality comparison
    ht.htsvd_set_basis(dn.ctx, 8, 3, *shipped[0])
    dn.denoise(d_in, AUTO, p_plain, out=d_out)
    psnr_shipped = synth.psnr(clean, d_out.cpu().numpy())
    n_vec, ops = gram_ops(h, w, c, s)
    tops = ops / (ms_gram * 1e-3) / 1e12
    log("learned basis: step %.2f ms, learn %.2f ms, Gram kernel %.3f ms, PSNR %.3f (shipped basis %.3f)"
        % (ms_step, learn_ms, ms_gram, psnr_learned, psnr_shipped))
    result = {
        "metric": "Mpixel/s denoised with a basis learned from the image itself, 12MP RGB sigma=50",
        "value": round(h * w / (ms_step * 1e-3) / 1e6, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32+f32",
        "data": "synthetic",
        "config": {"workload": "12MP RGB %dx%d, AWGN sigma=%g estimated (plain estimator + vote), basis learned "
                               "from the noisy image (reference stride %d), ps 8, window %d, K 32"
                               % (w, h, sigma, s, p_plain.window), "form": "plain + learned basis"},
        "learn_ms": round(learn_ms, 3),
        "roofline": {"bound": "alu", "kernel": "gram_kernel<3>", "achieved": round(tops, 3),
                     "peak": PEAK_INT32_VALU_TOPS, "unit": "TOP/s", "frac": round(tops / PEAK_INT32_VALU_TOPS, 4),
                     "traffic": measured_traffic(n_vec, GRAM_TRAFFIC_FILE, GRAM_SRC, "src_sha256_16", "vectors"),
                     "kernel_ms": round(ms_gram, 4), "ops_per_launch": ops, "vectors": n_vec},
        "psnr": {"learned_basis": round(psnr_learned, 3), "shipped_basis": round(psnr_shipped, 3)},
        "input_gen_s": round(gen_s, 1),
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline_learn(noisy, s, args.cpu_seconds)
    print(json.dumps(result), flush=True)


def cpu_baseline_learn(noisy, s, target_s):
    """The oracle's learning (FFT of the patches, covariances, eigh) on a top band of the image,
    scaled to pixels of the band."""
    from oracle import learn_basis as lb
    t0 = time.time()
    band = noisy[:64]
    lb.learn(band, 8, s)
    t1 = time.time() - t0
    rows = int(min(noisy.shape[0], max(64, 64 * target_s / max(t1, 1e-3))))
    band = noisy[:rows]
    t0 = time.time()
    lb.learn(band, 8, s)
    dt = time.time() - t0
    return {"value": round(band.shape[0] * band.shape[1] / dt / 1e6, 5), "unit": "Mpixel/s", "cores": 1,
            "kind": "oracle", "sample": "the top %d rows of the same image (%.1f s), oracle learning only" % (rows, dt)}


def cpu_baseline(noisy, s, W, K, sigma, target_s):
    """The FP64 oracle, as it stands, on a band of reference rows of the same image (known
    sigma: the oracle's filter, the dominant cost of the path)."""
    import oracle
    h, w = noisy.shape[:2]
    ny, nx = oracle.n_refs(h, w, 8, s)
    U, V = oracle.load_basis(os.path.join(ROOT, "paper_2512_23569_amd", "data", "basis_ps8_c3.f64"), 8, 3)
    tau = sigma * oracle.tau_multiplier(3, K)
    cores = os.cpu_count() or 1
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        pass
    # probe with eight reference rows (enough work for every core), then size the sample to
    # about target_s seconds
    t0 = time.time()
    oracle.denoise(noisy, U, V, tau, s=s, W=W, K=K, nthreads=cores, r_begin=0, r_end=8 * nx)
    t1 = (time.time() - t0) / 8
    rows = max(1, min(ny, int(target_s / max(t1, 1e-3))))
    log("cpu oracle: %.3f s per row, sampling %d rows" % (t1, rows))
    t0 = time.time()
    oracle.denoise(noisy, U, V, tau, s=s, W=W, K=K, nthreads=cores, r_begin=0, r_end=rows * nx)
    dt = time.time() - t0
    n = rows * nx
    # each reference stands for stride^2 pixels of the grid
    mpx_s = n * s * s / dt / 1e6
    # one thread, on a sample of about a third of the target time
    rows1 = max(1, min(ny, int(target_s / 3.0 / max(t1 * cores, 1e-3))))
    t0 = time.time()
    oracle.denoise(noisy, U, V, tau, s=s, W=W, K=K, nthreads=1, r_begin=0, r_end=rows1 * nx)
    dt1 = time.time() - t0
    log("cpu oracle, one thread: %d rows in %.1f s" % (rows1, dt1))
    return {"value": round(mpx_s, 5), "unit": "Mpixel/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "%d reference rows (%d references, %.1f s) of the same 12 MP image, FP64 oracle, known sigma"
                      % (rows, n, dt),
            "single_thread": {"value": round(rows1 * nx * s * s / dt1 / 1e6, 5), "unit": "Mpixel/s", "cores": 1,
                              "sample": "%d reference rows (%.1f s)" % (rows1, dt1)}}


if __name__ == "__main__":
    main()
