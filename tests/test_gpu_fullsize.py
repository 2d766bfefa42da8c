"""Parity at the full workload sizes (needs an MI355X).

Workloads: the 12 MP RGB image the benchmark times (textured, AWGN sigma 50, reference stride
3, window 31, K = 32, noise level estimated) in its plain form (plain estimator and the Eq. 23
vote) and its batched + learned form (learned map judged by the plain estimate, the vote,
HTSVD_K_AUTO, graph replay); the same image with Poisson-Gaussian noise; and the 64-image
batch.  The FP64 oracle cannot denoise 12 MP within a test, so it checks what it can compute
exactly:

  - groups of sampled references, bit-exact (indices and distances), including the last
    reference row and column of the grid;
  - sigma_est of sampled sub-images (relative 1e-9), including partial edge sub-images, and
    their Eq. 23 votes (identical counts), from oracle groups of the sampled voters;
  - denoised pixels of row bands: the oracle processes every reference whose groups can reach
    the band (reference rows within R + ps - 1 of it), so the band's pixels are complete sums,
    with thresholds from its own estimates and votes of every sub-image those references lie in
    (and, for the learned form, the oracle rule applied to the GPU's map); the pixel parity bar
    (>= 99.99% within 1e-2, |dPSNR| <= 0.01 dB) applies to each band;
  - the guard band's overflow counter (near-threshold coefficients decided in FP32) is zero.

The video workload the benchmark times (7 frames of 1080 x 1920 RGB, AWGN sigma 30, temporal
radius 1, stride 4, window 15, K 32) is checked the same way: all spatio-temporal groups
bit-exact (the oracle matches the whole clip in seconds), and row bands of three frames (top,
middle, bottom) denoised by the oracle from every group with a member patch in the band.
"""
import os

import numpy as np
import pytest

import oracle
import synth
from helpers import PIX_FRAC, PIX_TOL
from oracle import estimator as est

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PS, S, W, K = 8, 3, 31, 32


@pytest.fixture(scope="module")
def dn():
    import paper_2512_23569_amd as ht
    assert torch.cuda.is_available(), "GPU tests need a device"
    d = ht.Denoiser(0, load_network=False)
    yield d
    d.close()


@pytest.fixture(scope="module")
def big():
    clean, noisy, spec = synth.make_cfg("rgb12mp_pg")
    return clean, noisy


@pytest.fixture(scope="module")
def bench_img():
    """The benchmark's own input: the 12 MP textured image (seed 3) with AWGN sigma 50 (seed 1003)."""
    clean = synth.make_clean(3000, 4000, 3, seed=3, texture=True)
    return clean, synth.add_awgn(clean, 50.0, seed=1003)


@pytest.fixture(scope="module")
def bench_sigma(bench_img):
    """Oracle plain estimates and Eq. 23 votes (32-member oracle groups of the sampled voters) of
    every sub-image of the benchmark input: shared by its plain and batched + learned forms."""
    clean, noisy = bench_img
    h, w = noisy.shape[:2]
    sp = est.sigma_est_tiles(noisy)
    ys, xs = oracle.ref_grid(h, PS, S), oracle.ref_grid(w, PS, S)
    tile_of = est.tile_of_refs(ys, xs, h, w)
    nty, ntx = est.tile_grid(h, w)
    votes = np.zeros(nty * ntx, dtype=np.int64)
    nvotes = np.zeros(nty * ntx, dtype=np.int64)
    voters = [est.vote_samples(np.nonzero(tile_of == t)[0], t) for t in range(nty * ntx)]
    gi, _ = oracle.block_match_list(noisy, np.concatenate(voters), PS, S, W, K)
    k = 0
    for t, v in enumerate(voters):
        votes[t] = sum(est.rank_position(est.group_vectors(noisy, gi[k + i], PS)) <= 13 for i in range(len(v)))
        nvotes[t] = len(v)
        k += len(v)
    return sp, (votes, nvotes)


def _ref_rows_for_band(h, y0, y1, s=S, w=W):
    """Reference-row range [a, b) whose groups can reach pixel rows [y0, y1)."""
    R = (w - 1) // 2
    ys = oracle.ref_grid(h, PS, s)
    keep = np.nonzero((ys >= y0 - (PS - 1) - R) & (ys <= y1 - 1 + R))[0]
    return int(keep[0]), int(keep[-1]) + 1


def _tiles_of_ref_rows(h, w, a, b, s=S):
    """Sub-images holding the top-left pixels of the references in grid rows [a, b)."""
    ys = oracle.ref_grid(h, PS, s)
    nty, ntx = est.tile_grid(h, w)
    rows = sorted(set(int(y) // 128 for y in ys[a:b]))
    return [r * ntx + t for r in rows for t in range(ntx)]


def _band_parity(gpu, ref, clean, y0, y1):
    g = gpu[y0:y1].astype(np.float64)
    r = ref[y0:y1]
    d = np.abs(g - r)
    frac = float(np.mean(d <= PIX_TOL))
    dps = abs(synth.psnr(clean[y0:y1], g) - synth.psnr(clean[y0:y1], r))
    assert frac >= PIX_FRAC and dps <= 0.01, (y0, y1, frac, float(d.max()), dps)
    return frac, float(d.max()), dps


# guard band of the filter: near-threshold coefficients beyond the per-group FP64 list are decided
# in FP32; at 12 MP (1.33 M groups) none is expected and none is allowed
GUARD_OVERFLOW_MAX = 0


@pytest.mark.parametrize("which", ["pg", "bench"])
def test_12mp_groups_sampled_bitexact(dn, big, bench_img, which):
    clean, noisy = big if which == "pg" else bench_img
    h, w = noisy.shape[:2]
    p = dn.params(3, stride=S, window=W, K=K)
    idx, dist = dn.block_match(torch.from_numpy(noisy).cuda(), p)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    ny, nx = oracle.n_refs(h, w, PS, S)
    rng = np.random.default_rng(12)
    refs = np.concatenate([rng.integers(0, ny * nx, 3000), np.arange((ny - 1) * nx, ny * nx, 37),
                           np.arange(nx - 1, ny * nx, nx * 29), [0, nx - 1, ny * nx - 1]])
    oi, od = oracle.block_match_list(noisy, refs, PS, S, W, K)
    bad = np.nonzero(np.any(idx[refs] != oi, axis=1) | np.any(dist[refs] != od, axis=1))[0]
    assert bad.size == 0, "reference %d: gpu %s oracle %s" % (refs[bad[0]], idx[refs[bad[0]]], oi[bad[0]])


def test_12mp_sigma_and_votes_sampled(dn, big):
    import paper_2512_23569_amd as ht
    clean, noisy = big
    h, w = noisy.shape[:2]
    p = dn.params(3, stride=S, window=W, K=K, adaptive=1)
    nty, ntx = est.tile_grid(h, w, 128)
    se = torch.zeros(nty * ntx, dtype=torch.float64, device="cuda")
    sh = torch.zeros_like(se)
    votes = torch.zeros(nty * ntx, dtype=torch.int32, device="cuda")
    x = torch.from_numpy(noisy).cuda()
    ht.htsvd_estimate_sigma(dn.ctx, x, h, w, 3, x.stride(0), -1.0, p, se, sh, votes)
    se, sh, votes = se.cpu().numpy(), sh.cpu().numpy(), votes.cpu().numpy()
    rng = np.random.default_rng(13)
    tiles = sorted(set(rng.integers(0, nty * ntx, 16).tolist()) | {0, ntx - 1, (nty - 1) * ntx, nty * ntx - 1})
    ref_se = est.sigma_est_tiles(noisy, tiles=tiles)
    assert np.allclose(se[tiles], ref_se[tiles], rtol=1e-9, atol=0), (se[tiles], ref_se[tiles])
    # votes of the sampled tiles from oracle groups of the sampled voters
    ys, xs = oracle.ref_grid(h, PS, S), oracle.ref_grid(w, PS, S)
    tile_of = est.tile_of_refs(ys, xs, h, w, 128)
    for t in tiles:
        voters = est.vote_samples(np.nonzero(tile_of == t)[0], t, p.n_vote, p.vote_seed)
        gi, _ = oracle.block_match_list(noisy, voters, PS, S, W, K)
        yes = sum(est.rank_position(est.group_vectors(noisy, gi[i], PS)) <= p.gamma_rank for i in range(len(voters)))
        assert votes[t] == yes, (t, votes[t], yes)
        want = ref_se[t] / p.beta if 2 * yes > len(voters) else ref_se[t]
        assert np.isclose(sh[t], want, rtol=1e-9, atol=0), (t, sh[t], want)


BANDS = ((1504, 1552), (3000 - 40, 3000))


def _oracle_bands(noisy, out, clean, tau_of_tiles, K_used, U, V):
    """Oracle denoising of every reference whose groups reach each band, with the thresholds
    tau_of_tiles(tiles) returns (oracle arithmetic only), then the pixel parity bar per band."""
    h, w = noisy.shape[:2]
    ny, nx = oracle.n_refs(h, w, PS, S)
    res = []
    for y0, y1 in BANDS:
        a, b = _ref_rows_for_band(h, y0, y1)
        tau = tau_of_tiles(_tiles_of_ref_rows(h, w, a, b))
        band = tau[a * nx:b * nx]
        assert np.all(np.isfinite(band)) and np.all(band > 0)
        tau = np.where(np.isfinite(tau), tau, 0.0)
        ref = oracle.denoise(noisy, U, V, tau, s=S, W=W, K=K_used, r_begin=a * nx, r_end=b * nx)
        res.append(_band_parity(out, ref, clean, y0, y1))
    return res


def test_12mp_plain_form_bands(dn, bench_img, bench_sigma, basis3):
    """The benchmark's plain form (AWGN sigma 50 estimated by the plain estimator with the vote,
    K = 32) against the oracle on two row bands; the oracle's thresholds come from its own
    estimates and votes of the sub-images the bands' references lie in."""
    clean, noisy = bench_img
    sp, votes = bench_sigma
    p = dn.params(3, stride=S, window=W, K=K, adaptive=1, estimator=0)
    x = torch.from_numpy(noisy).cuda()
    out = dn.denoise(x, -1.0, p).cpu().numpy()
    guard = dn.guard_count()
    assert guard[1] <= GUARD_OVERFLOW_MAX, guard
    U, V = basis3
    res = _oracle_bands(noisy, out, clean, lambda tiles: est.thresholds(
        noisy, PS, S, W, K, tiles=tiles, sigma_plain=sp, votes=votes)["tau"], K, U, V)
    print("plain form: guard %s, bands %s" % (guard, res))


def test_12mp_ra_form_bands(dn, bench_img, bench_sigma, basis3):
    """The benchmark's RA-Haar-tSVD form (the plain form with the shipped refinement network,
    every group above sigma 30 refined) against the oracle on two row bands: oracle groups and
    mean patches, the FP64 network, the oracle's own thresholds."""
    import paper_2512_23569_amd as ht
    from oracle import fcn
    path = os.path.join(ht.DATA_DIR, "ra_fcn_c3.f32")
    if not os.path.exists(path):
        pytest.skip("no trained RA network shipped")
    w32 = np.fromfile(path, dtype="<f4")
    ht.htsvd_ra_set_weights(dn.ctx, 3, w32)
    clean, noisy = bench_img
    h, w = noisy.shape[:2]
    sp, votes = bench_sigma
    p = dn.params(3, stride=S, window=W, K=K, adaptive=1, estimator=0, ra=1)
    out = dn.denoise(torch.from_numpy(noisy).cuda(), -1.0, p).cpu().numpy()
    guard = dn.guard_count()
    assert guard[1] <= GUARD_OVERFLOW_MAX, guard
    U, V = basis3
    ny, nx = oracle.n_refs(h, w, PS, S)
    m = oracle.tau_multiplier(3, K)
    res = []
    for y0, y1 in BANDS:
        a, b = _ref_rows_for_band(h, y0, y1)
        tau = est.thresholds(noisy, PS, S, W, K, tiles=_tiles_of_ref_rows(h, w, a, b), sigma_plain=sp,
                             votes=votes)["tau"]
        refs = np.arange(a * nx, b * nx)
        assert np.all(np.isfinite(tau[refs])) and np.all(tau[refs] > 0)
        tau = np.where(np.isfinite(tau), tau, 0.0)
        gi, _ = oracle.block_match_list(noisy, refs, PS, S, W, K)
        pest = np.zeros((ny * nx, 3 * PS * PS))
        pest[refs] = fcn.refine(w32.astype(np.float64), fcn.group_means(noisy, gi).reshape(len(refs), -1), 3)
        ra_on = np.zeros(ny * nx, dtype=bool)
        ra_on[refs] = tau[refs] / m > 30.0
        ref = oracle.denoise(noisy, U, V, tau, s=S, W=W, K=K, r_begin=a * nx, r_end=b * nx, pest=pest, ra_on=ra_on)
        res.append(_band_parity(out, ref, clean, y0, y1) + (int(ra_on[refs].sum()), len(refs)))
    print("RA form: guard %s, bands (frac, max, dPSNR, refined, refs) %s" % (guard, res))


def test_12mp_batched_learned_form_bands(dn, bench_img, bench_sigma, basis3):
    """The benchmark's batched + learned form (one-image batch through the graph, learned map,
    vote, HTSVD_K_AUTO at the autotuner's cutoff) against the oracle: the group size the device
    chose, and two row bands with the oracle rule's thresholds (the GPU's map z given to it)."""
    import paper_2512_23569_amd as ht
    if not os.path.exists(os.path.join(ht.DATA_DIR, "sigma_cnn_c3.ckpt")):
        pytest.skip("no trained network shipped")
    clean, noisy = bench_img
    h, w = noisy.shape[:2]
    sp, votes = bench_sigma
    d = ht.Denoiser(0)
    try:
        x = torch.from_numpy(noisy).cuda()
        z = d.sigma_map(x).cpu().numpy()
        cutoff = 77.5    # the autotuner's cutoff on its calibration images (K = 16 never loses there)
        p = d.params(3, stride=S, window=W, K=K, adaptive=1, estimator=1)
        out = d.denoise_batch([x], [-1.0], p, Ks=[ht.HTSVD_K_AUTO], use_graph=True, k_sigma_cutoff=cutoff)
        out = d.denoise_batch([x], [-1.0], p, outs=out, Ks=[ht.HTSVD_K_AUTO], use_graph=True,
                              k_sigma_cutoff=cutoff)[0].cpu().numpy()
        pre = est.thresholds(noisy, PS, S, W, K, z=z, sigma_plain=sp, adaptive=False)
        m32 = oracle.tau_multiplier(3, 32)
        K_used = est.auto_group_size(pre["tau"] / m32, cutoff)
        assert ht.htsvd_batch_inspect(d.ctx, 0) == K_used
        tau_gpu = torch.zeros(pre["tau"].size, dtype=torch.float64, device="cuda")
        ht.htsvd_batch_inspect(d.ctx, 0, tau_gpu)
        tg = tau_gpu.cpu().numpy()
        ys, xs = oracle.ref_grid(h, PS, S), oracle.ref_grid(w, PS, S)
        tile_of = est.tile_of_refs(ys, xs, h, w)
        ny, nx = oracle.n_refs(h, w, PS, S)
        def tau_of_tiles(tiles):
            # the vote of the sampled tiles on groups of the chosen size (the first K_used members)
            votes_k = votes if K_used == 32 else None
            r = est.thresholds(noisy, PS, S, W, K_used, z=z, sigma_plain=sp, votes=votes_k, tiles=tiles)
            sel = np.isfinite(r["tau"])
            keep_ref = ~r["use_plain"][tile_of[sel]]
            tol = np.where(keep_ref, 1e-12, 1e-9)
            assert np.all(np.abs(tg[sel] - r["tau"][sel]) <= tol * r["tau"][sel]), \
                float(np.max(np.abs(tg[sel] - r["tau"][sel]) / r["tau"][sel]))
            return r["tau"]

        U, V = basis3
        res = _oracle_bands(noisy, out, clean, tau_of_tiles, K_used, U, V)
        print("batched + learned: K %d, bands %s" % (K_used, res))
    finally:
        d.close()


def test_batch_of_64_sampled_bands(dn, basis3):
    """The 64-image batch through one graph replay (known per-image sigma, K = 16 as the
    autotuner picks for it): bands of the largest and smallest images against the oracle."""
    specs = synth.batch_specs(64, seed=4)
    pairs = [(synth.make_clean(hh, ww, 3, sd), hh, ww, sg, sd) for hh, ww, sg, sd in specs]
    noisy = [synth.add_awgn(c, sg, sd + 1000) for c, hh, ww, sg, sd in pairs]
    ins = [torch.from_numpy(n).cuda() for n in noisy]
    sig = [sp[2] for sp in specs]
    p = dn.params(3, stride=4, window=31, K=16)
    outs = dn.denoise_batch(ins, sig, p, use_graph=True)
    outs = dn.denoise_batch(ins, sig, p, outs=outs, use_graph=True)   # replay
    torch.cuda.synchronize()
    U, V = basis3
    sizes = [n.shape[0] * n.shape[1] for n in noisy]
    for i in (int(np.argmax(sizes)), int(np.argmin(sizes))):
        h, w = noisy[i].shape[:2]
        ny, nx = oracle.n_refs(h, w, PS, 4)
        tau = sig[i] * oracle.tau_multiplier(3, 16)
        y0, y1 = h // 2 - 16, h // 2 + 16
        a, b = _ref_rows_for_band(h, y0, y1, s=4)
        ref = oracle.denoise(noisy[i], U, V, tau, s=4, W=31, K=16, r_begin=a * nx, r_end=b * nx)
        _band_parity(outs[i].cpu().numpy(), ref, pairs[i][0], y0, y1)


def test_video_full_size_groups_and_bands(dn):
    import os
    T, h, w, c, sigma, radius, Kv, Wv, sv = 7, 1080, 1920, 3, 30.0, 1, 32, 15, 4
    clean = synth.make_video(T, h, w, c, seed=21)
    noisy = synth.add_awgn(clean, sigma, seed=22)
    d = torch.from_numpy(noisy).cuda()
    p = dn.params(c, stride=sv, window=Wv, K=Kv)
    gi, gd = dn.block_match_video(d, p, radius)
    gpu = dn.denoise_video(d, sigma, p, radius).cpu().numpy()
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    oi, od = oracle.block_match_video(noisy, PS, sv, Wv, Kv, radius)
    assert np.array_equal(gd, od)
    assert np.array_equal(gi, oi)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    U, V = oracle.load_basis(os.path.join(root, "paper_2512_23569_amd", "data", "basis_ps8_c3.f64"), 8, 3)
    tau = sigma * oracle.tau_multiplier(c, Kv)
    stacked = noisy.reshape(T * h, w, c)
    frame, row = oi // (h * w), (oi % (h * w)) // w
    for t, y0, y1 in ((3, 0, 32), (0, 520, 552), (6, h - 32, h)):
        hit = ((frame == t) & (row + PS - 1 >= y0) & (row <= y1 - 1)).any(axis=1)
        ref = oracle.filter_groups(stacked, oi[hit], U, V, tau, nthreads=4).reshape(T, h, w, c)
        _band_parity(gpu[t], ref[t], clean[t], y0, y1)
