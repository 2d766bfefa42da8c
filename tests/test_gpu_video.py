"""Video (Sec. IV-C) on the GPU vs the FP64 oracle (needs an MI355X): the spatio-temporal groups
bit-exact, and the denoised frames to the pixel parity bar."""
import os

import numpy as np
import pytest

import oracle
import synth
from helpers import assert_pixel_parity
from oracle import fcn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dn():
    import paper_2512_23569_amd as ht
    assert torch.cuda.is_available(), "GPU tests need a device"
    d = ht.Denoiser(0, load_network=False)
    yield d
    d.close()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _tie_heavy_video(T, h, w, c, seed):
    rng = np.random.default_rng(seed)
    v = (rng.integers(0, 4, (T, h, w, c) if c == 3 else (T, h, w)) * 60).astype(np.uint8)
    v[:, : h // 5] = 0
    v[1] = v[0]                                   # equal distances in two frames
    v[-1, 10:18, 12:20] = v[0, 3:11, 5:13]        # moved content
    return v


# (T, h, w, c, K, W, s, radius): ragged frame sizes, every group size, the widest window,
# a radius beyond the video's length, a single frame
CASES = [(3, 40, 48, 3, 16, 15, 4, 1), (5, 37, 45, 1, 8, 21, 3, 2), (2, 64, 72, 3, 32, 31, 4, 1),
         (4, 33, 41, 3, 4, 9, 5, 3), (3, 30, 38, 1, 32, 13, 2, 5), (1, 48, 40, 3, 16, 15, 4, 2)]


@pytest.mark.parametrize("T,h,w,c,K,W,s,radius", CASES)
def test_video_groups_exact(dn, T, h, w, c, K, W, s, radius):
    v = synth.add_awgn(synth.make_video(T, h, w, c, 100 + T + h), 25.0, 101 + w)
    idx, dist = dn.block_match_video(_dev(v), dn.params(c, stride=s, window=W, K=K), radius)
    torch.cuda.synchronize()
    oi, od = oracle.block_match_video(v, 8, s, W, K, radius)
    assert np.array_equal(dist.cpu().numpy(), od)
    assert np.array_equal(idx.cpu().numpy(), oi)


@pytest.mark.parametrize("c,radius", [(3, 1), (1, 2)])
def test_video_groups_exact_with_ties(dn, c, radius):
    v = _tie_heavy_video(4, 36, 44, c, 110 + c)
    idx, dist = dn.block_match_video(_dev(v), dn.params(c, stride=3, window=13, K=16), radius)
    torch.cuda.synchronize()
    oi, od = oracle.block_match_video(v, 8, 3, 13, 16, radius)
    assert np.array_equal(dist.cpu().numpy(), od)
    assert np.array_equal(idx.cpu().numpy(), oi)


def test_video_radius_zero_equals_the_image_matcher(dn):
    v = synth.add_awgn(synth.make_video(3, 44, 52, 3, 120), 20.0, 121)
    p = dn.params(3, stride=4, window=15, K=16)
    iv, dv = dn.block_match_video(_dev(v), p, 0)
    per = iv.shape[0] // 3
    for t in range(3):
        i, d = dn.block_match(_dev(v[t]), p)
        torch.cuda.synchronize()
        assert torch.equal(iv[t * per:(t + 1) * per], i + t * 44 * 52)
        assert torch.equal(dv[t * per:(t + 1) * per], d)


# The filter adds each tile's patches into LDS regions of the frames a tile can reach (tile side 4,
# 3 with a wider window and radius) and falls back to direct global sums when they do not fit
# (11 frames within radius 5 at window 31).
@pytest.mark.parametrize("T,h,w,c,K,W,radius,sigma", [(4, 48, 56, 3, 16, 15, 1, 30.0), (3, 40, 44, 1, 8, 13, 1, 25.0),
                                                      (5, 36, 40, 3, 32, 13, 2, 40.0), (2, 41, 37, 3, 4, 9, 1, 15.0),
                                                      (5, 44, 52, 3, 16, 21, 2, 30.0), (11, 40, 48, 3, 32, 31, 5, 35.0),
                                                      (6, 38, 46, 1, 16, 31, 5, 25.0)])
def test_video_denoise_parity(dn, T, h, w, c, K, W, radius, sigma):
    clean = synth.make_video(T, h, w, c, 130 + T)
    noisy = synth.add_awgn(clean, sigma, 131 + T)
    U, V = oracle.load_basis(os.path.join(ROOT, "paper_2512_23569_amd", "data", "basis_ps8_c%d.f64" % c), 8, c)
    idx, _ = oracle.block_match_video(noisy, 8, 4, W, K, radius)
    tau = sigma * oracle.tau_multiplier(c, K)
    stacked = noisy.reshape((T * h, w) + noisy.shape[3:])
    ref = oracle.filter_groups(stacked, idx, U, V, tau).reshape(noisy.shape)
    p = dn.params(c, stride=4, window=W, K=K)
    gpu = dn.denoise_video(_dev(noisy), sigma, p, radius).cpu().numpy()
    m = assert_pixel_parity(gpu, ref, clean)
    print("video T=%d c=%d K=%d radius=%d sigma=%g" % (T, c, K, radius, sigma), m)
    assert m["psnr_gpu"] > synth.psnr(clean, noisy) + 1.0   # small, textured clips: a modest gain


def test_video_follows_the_installed_basis(dn):
    """The filter's FP64 maps are rebuilt when the basis changes (here: learned from the video)."""
    import paper_2512_23569_amd as ht
    T, h, w, c, sigma = 3, 40, 48, 3, 30.0
    clean = synth.make_video(T, h, w, c, 140)
    noisy = synth.add_awgn(clean, sigma, 141)
    p = dn.params(c, stride=4, window=13, K=16)
    first = dn.denoise_video(_dev(noisy), sigma, p, 1).cpu().numpy()
    stacked = noisy.reshape(T * h, w, c)
    U, V = dn.learn_basis(_dev(stacked), stride=4)
    second = dn.denoise_video(_dev(noisy), sigma, p, 1).cpu().numpy()
    idx, _ = oracle.block_match_video(noisy, 8, 4, 13, 16, 1)
    ref = oracle.filter_groups(stacked, idx, oracle.from_slices(U), oracle.from_slices(V),
                               sigma * oracle.tau_multiplier(c, 16)).reshape(noisy.shape)
    assert_pixel_parity(second, ref, clean)
    assert np.abs(first - second).max() > 0.5
    # the shipped basis again
    Us, Vs = oracle.load_basis(os.path.join(ROOT, "paper_2512_23569_amd", "data", "basis_ps8_c3.f64"), 8, 3)
    ht.htsvd_set_basis(dn.ctx, 8, 3, oracle.to_slices(Us), oracle.to_slices(Vs))
    third = dn.denoise_video(_dev(noisy), sigma, p, 1).cpu().numpy()
    assert np.array_equal(third, first)


def test_video_radius_zero_matches_the_image_denoiser(dn):
    """Radius 0 groups each frame alone, so every frame is the image denoiser's output up to the
    rounding of the two aggregations (fixed point at 2^-12 here, 2^-9 or finer per tile there)."""
    T, h, w = 3, 44, 52
    noisy = synth.add_awgn(synth.make_video(T, h, w, 3, 150), 30.0, 151)
    p = dn.params(3, stride=4, window=13, K=16)
    vid = dn.denoise_video(_dev(noisy), 30.0, p, 0).cpu().numpy()
    for t in range(T):
        img = dn.denoise(_dev(noisy[t]), 30.0, p).cpu().numpy()
        assert np.abs(vid[t] - img).max() <= 4e-3


def _ra_weights(c, seed):
    p = fcn.init_params(c, seed) * 0.3
    rng = np.random.default_rng(seed + 100)
    p = p + rng.normal(0, 0.01, p.size) * (p != 0)
    o = 0
    for sh in fcn.shapes(c):
        n = int(np.prod(sh))
        if len(sh) == 1:
            p[o:o + n] = rng.normal(0, 0.05, n)
        o += n
    return p.astype(np.float32)


@pytest.mark.parametrize("c,K,sigma,radius", [(3, 16, 50.0, 1), (1, 8, 45.0, 2), (3, 32, 60.0, 1)])
def test_video_ra_parity(dn, c, K, sigma, radius):
    """RA-Haar-tSVD on the spatio-temporal groups: oracle groups, oracle mean patches, the FP64
    network and the FP64 groups filter with the refined first Haar row."""
    import paper_2512_23569_amd as ht
    wts = _ra_weights(c, 30 + K)
    ht.htsvd_ra_set_weights(dn.ctx, c, wts)
    T, h, w = 3, 40, 48
    clean = synth.make_video(T, h, w, c, 160 + K)
    noisy = synth.add_awgn(clean, sigma, 161 + K)
    stacked = noisy.reshape((T * h, w) + noisy.shape[3:])
    U, V = oracle.load_basis(os.path.join(ROOT, "paper_2512_23569_amd", "data", "basis_ps8_c%d.f64" % c), 8, c)
    idx, _ = oracle.block_match_video(noisy, 8, 4, 13, K, radius)
    pest = fcn.refine(wts.astype(np.float64), fcn.group_means(stacked, idx).reshape(len(idx), -1), c)
    tau = sigma * oracle.tau_multiplier(c, K)
    ref = oracle.filter_groups(stacked, idx, U, V, tau, pest=pest).reshape(noisy.shape)
    p = dn.params(c, stride=4, window=13, K=K, ra=1)
    gpu = dn.denoise_video(_dev(noisy), sigma, p, radius).cpu().numpy()
    m = assert_pixel_parity(gpu, ref, clean)
    plain = oracle.filter_groups(stacked, idx, U, V, tau).reshape(noisy.shape)
    print("video RA c=%d K=%d sigma=%g" % (c, K, sigma), m, "mean |RA - plain| %.3f" % np.abs(ref - plain).mean())
    assert np.abs(ref - plain).mean() > 0.1


@pytest.mark.parametrize("c,sigma,known", [(3, 40.0, False), (1, 30.0, True)])
def test_video_adaptive_parity(dn, c, sigma, known):
    """A-Haar-tSVD frame by frame (Sec. IV-C): each frame's sub-image noise estimate (or the known
    sigma) adjusted by the vote over the frame's spatial groups (Eq. 22-23) sets the thresholds of
    its references; the spatio-temporal groups are filtered with them."""
    from oracle import estimator as est
    T, h, w, K, W, s, radius = 3, 136, 160, 16, 15, 4, 1
    clean = synth.make_video(T, h, w, c, 170 + c)
    noisy = synth.add_awgn(clean, sigma, 171 + c)
    p = dn.params(c, stride=s, window=W, K=K, adaptive=1)
    gpu = dn.denoise_video(_dev(noisy), sigma if known else -1.0, p, radius).cpu().numpy()
    U, V = oracle.load_basis(os.path.join(ROOT, "paper_2512_23569_amd", "data", "basis_ps8_c%d.f64" % c), 8, c)
    taus = []
    for t in range(T):
        it, _ = oracle.block_match(noisy[t], 8, s, W, K)
        start = np.full(4, sigma) if known else est.sigma_est_tiles(noisy[t])
        sig = est.sigma_hat_tiles(noisy[t], it, start, 8, s)
        taus.append(est.tau_per_ref(sig, h, w, 8, s, c, K))
    idx, _ = oracle.block_match_video(noisy, 8, s, W, K, radius)
    stacked = noisy.reshape((T * h, w) + noisy.shape[3:])
    ref = oracle.filter_groups(stacked, idx, U, V, np.concatenate(taus)).reshape(noisy.shape)
    m = assert_pixel_parity(gpu, ref, clean)
    print("video adaptive c=%d sigma=%g known=%s" % (c, sigma, known), m)


def test_video_learned_estimator_frame_by_frame():
    """The learned noise estimator runs frame by frame: at radius 0 every frame is the image
    denoiser's output with the same estimator (up to the aggregations' rounding)."""
    import paper_2512_23569_amd as ht
    d = ht.Denoiser(0)
    try:
        T, h, w = 2, 136, 152
        noisy = synth.add_awgn(synth.make_video(T, h, w, 3, 180), 35.0, 181)
        p = d.params(3, stride=4, window=15, K=16, estimator=1, adaptive=1)
        vid = d.denoise_video(_dev(noisy), ht.HTSVD_SIGMA_AUTO, p, 0).cpu().numpy()
        for t in range(T):
            img = d.denoise(_dev(noisy[t]), ht.HTSVD_SIGMA_AUTO, p).cpu().numpy()
            assert np.abs(vid[t] - img).max() <= 4e-3
    finally:
        d.close()


def test_video_padded_strides_through_the_c_abi(dn):
    """Row strides wider than the frames, for the input and the output, through the C entry
    points: the same groups and the same output bit for bit as the contiguous call."""
    import paper_2512_23569_amd as ht
    T, h, w, c, radius = 3, 40, 44, 3, 1
    v = synth.add_awgn(synth.make_video(T, h, w, c, 190), 30.0, 191)
    p = dn.params(c, stride=4, window=13, K=16)
    idx, dist = dn.block_match_video(_dev(v), p, radius)
    out = dn.denoise_video(_dev(v), 30.0, p, radius)
    in_stride, out_stride = w * c + 20, w * c + 9
    padded = np.full((T * h, in_stride), 7, np.uint8)
    padded[:, :w * c] = v.reshape(T * h, w * c)
    d_pad = _dev(padded)
    n_ref = idx.shape[0]
    idx2 = torch.empty((n_ref, 16), dtype=torch.int32, device="cuda")
    dist2 = torch.empty((n_ref, 16), dtype=torch.int32, device="cuda")
    ht.htsvd_block_match_video(dn.ctx, d_pad, T, h, w, c, in_stride, radius, p, idx2, dist2)
    out2 = torch.full((T * h, out_stride), -5.0, dtype=torch.float32, device="cuda")
    ht.htsvd_denoise_video(dn.ctx, d_pad, T, h, w, c, in_stride, radius, 30.0, p, out2, out_stride)
    torch.cuda.synchronize()
    assert torch.equal(idx, idx2) and torch.equal(dist, dist2)
    assert torch.equal(out.reshape(T * h, w * c), out2[:, :w * c])
    assert torch.all(out2[:, w * c:] == -5.0)   # the padding of the output is not written


def test_video_errors(dn):
    import paper_2512_23569_amd as ht
    v = _dev(synth.make_video(2, 32, 32, 3, 160))
    p = dn.params(3, stride=4, window=13, K=16)
    with pytest.raises(ht.HtsvdError):
        dn.block_match_video(v, p, 32)                       # radius beyond 31
    with pytest.raises(ht.HtsvdError):
        dn.denoise_video(v, 30.0, p.replace(estimator=2), 1)  # no such estimator
    d2 = ht.Denoiser(0, load_network=False)
    try:
        with pytest.raises(ht.HtsvdError):                   # refinement without a network
            d2.denoise_video(v, 50.0, p.replace(ra=1), 1)
    finally:
        d2.close()
    with pytest.raises(ht.HtsvdError):
        dn.denoise_video(v, -2.0, p, 1)                      # neither a sigma nor AUTO
    with pytest.raises(ht.HtsvdError):                       # window too small for K
        dn.block_match_video(v, dn.params(3, stride=4, window=3, K=16), 1)
