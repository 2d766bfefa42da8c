"""Hyperspectral tube patches (Sec. IV-D) on the GPU vs the FP64 oracle (needs an MI355X): the
grouping guide and the groups bit-exact, the band t-product filter to the pixel parity bar."""
import numpy as np
import pytest

import oracle
import synth
from helpers import assert_pixel_parity
from oracle import learn_basis as lb

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dn():
    import paper_2512_23569_amd as ht
    assert torch.cuda.is_available(), "GPU tests need a device"
    d = ht.Denoiser(0, load_network=False)
    yield d
    d.close()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("bands", [2, 7, 31, 64])
def test_guide_and_groups_exact(dn, bands):
    cube = synth.add_awgn(synth.make_hsi(61, 70, bands, 80 + bands), 15.0, 81)
    g = dn.band_guide(_dev(cube))
    torch.cuda.synchronize()
    want = oracle.band_guide(cube)
    assert np.array_equal(g.cpu().numpy(), want)
    idx, dist = dn.block_match(g, dn.params(1, stride=4, window=15, K=16))
    oi, od = oracle.block_match(want, 8, 4, 15, 16)
    assert np.array_equal(idx.cpu().numpy(), oi) and np.array_equal(dist.cpu().numpy(), od)


# 32 bands fill the 32-wide band DFT of the kernel; 40 and 64 take the 64-wide one (two patches
# per workgroup); even band counts carry the real slice f = B/2
@pytest.mark.parametrize("bands,K,sigma,s", [(31, 16, 20.0, 4), (8, 8, 30.0, 3), (5, 32, 15.0, 4), (2, 4, 25.0, 2),
                                             (32, 16, 20.0, 4), (40, 8, 25.0, 4), (64, 4, 20.0, 4)])
def test_band_denoise_parity(dn, bands, K, sigma, s):
    import paper_2512_23569_amd as ht
    h, w = 56, 64
    clean = synth.make_hsi(h, w, bands, 90 + bands)
    noisy = synth.add_awgn(clean, sigma, 91 + bands)
    U, V = lb.learn(noisy, 8, 4)
    ht.htsvd_set_basis(dn.ctx, 8, bands, oracle.to_slices(U), oracle.to_slices(V))
    W = 15
    idx, _ = oracle.block_match(oracle.band_guide(noisy), 8, s, W, K)
    tau = sigma * np.sqrt(2.0 * np.log(bands * K * 64))
    ref = oracle.filter_groups(noisy, idx, U, V, tau)
    p = dn.params(1, stride=s, window=W, K=K)
    gpu = dn.denoise_bands(_dev(noisy), sigma, p).cpu().numpy()
    m = assert_pixel_parity(gpu, ref, clean)
    print("bands=%d K=%d sigma=%g" % (bands, K, sigma), m)
    assert m["psnr_gpu"] > synth.psnr(clean, noisy) + 3.0


def test_band_errors(dn):
    import paper_2512_23569_amd as ht
    d2 = ht.Denoiser(0, load_network=False)
    try:
        cube = _dev(synth.make_hsi(32, 32, 6, 95))
        with pytest.raises(ht.HtsvdError):   # no basis for 6 bands
            d2.denoise_bands(cube, 20.0, d2.params(1, stride=4, window=15, K=8))
        U, V = lb.learn(synth.make_hsi(32, 32, 6, 96), 8, 4)
        ht.htsvd_set_basis(d2.ctx, 8, 6, oracle.to_slices(U), oracle.to_slices(V))
        with pytest.raises(ht.HtsvdError):   # neither a sigma nor AUTO
            d2.denoise_bands(cube, -2.0, d2.params(1, stride=4, window=15, K=8))
        bad = oracle.to_slices(U).copy()
        bad[0, 0, 0] += 0.1
        with pytest.raises(ht.HtsvdError):   # not orthogonal
            ht.htsvd_set_basis(d2.ctx, 8, 6, bad, oracle.to_slices(V))
    finally:
        d2.close()


@pytest.mark.parametrize("bands,s", [(7, 4), (31, 3), (2, 5)])
def test_band_gram_sums_exact(dn, bands, s):
    cube = synth.add_awgn(synth.make_hsi(45, 52, bands, 100 + bands), 20.0, 101)
    G = dn.basis_gram(_dev(cube), stride=s)
    torch.cuda.synchronize()
    assert np.array_equal(G.cpu().numpy(), lb.channel_gram(cube, 8, s))


@pytest.mark.parametrize("bands", [5, 8, 31])
def test_band_learned_basis_and_denoise(dn, bands):
    """The basis learned on the GPU from the noisy cube (Sec. III-B with c = bands) matches the
    oracle's, and denoising with it matches oracle learning plus the oracle filter."""
    clean = synth.make_hsi(64, 56, bands, 110 + bands)
    noisy = synth.add_awgn(clean, 25.0, 111 + bands)
    d = _dev(noisy)
    Ug, Vg = dn.learn_basis(d, stride=4)
    Uo, Vo = lb.learn(noisy, 8, 4)
    du = np.abs(Ug - oracle.to_slices(Uo)).max()
    dv = np.abs(Vg - oracle.to_slices(Vo)).max()
    print("bands=%d max |dU| %.3g |dV| %.3g" % (bands, du, dv))
    assert du <= 1e-8 and dv <= 1e-8
    idx, _ = oracle.block_match(oracle.band_guide(noisy), 8, 4, 15, 16)
    ref = oracle.filter_groups(noisy, idx, Uo, Vo, 25.0 * np.sqrt(2.0 * np.log(bands * 16 * 64)))
    gpu = dn.denoise_bands(d, 25.0, dn.params(1, stride=4, window=15, K=16)).cpu().numpy()
    assert_pixel_parity(gpu, ref, clean)


@pytest.mark.parametrize("bands", [9, 40])
def test_band_filter_in_passes_is_identical(dn, bands):
    """A small memory cap splits the groups into several passes; the fixed-point aggregation
    makes the output identical to the single pass (the 32-wide and the 64-wide kernels)."""
    import paper_2512_23569_amd as ht
    noisy = synth.add_awgn(synth.make_hsi(72, 80, bands, 120), 20.0, 121)
    d = _dev(noisy)
    dn.learn_basis(d, stride=4)
    p = dn.params(1, stride=4, window=15, K=16)
    one = dn.denoise_bands(d, 20.0, p)
    ht.htsvd_set_band_memory(dn.ctx, 1 << 20)   # 1 MiB: 13 groups per pass at 9 bands, 3 at 40
    try:
        many = dn.denoise_bands(d, 20.0, p)
    finally:
        ht.htsvd_set_band_memory(dn.ctx, 4 << 30)
    torch.cuda.synchronize()
    assert torch.equal(one, many)


@pytest.mark.parametrize("h,w,bands", [(150, 140, 8), (64, 300, 5)])
def test_band_sigma_matches_oracle(dn, h, w, bands):
    """Band-wise noise levels (Sec. IV-D): the plain estimate of every band alone, averaged over
    its sub-images (partial edge sub-images included)."""
    levels = np.linspace(8.0, 30.0, bands)
    cube = synth.add_band_awgn(synth.make_hsi(h, w, bands, 110 + bands), levels, 111)
    got = dn.band_sigma(_dev(cube))
    want = oracle.band_sigma(cube)
    assert np.allclose(got, want, rtol=1e-9, atol=0), (got, want)


def test_band_sigma_full_size(dn):
    """The benchmark's band-wise workload at full size (512 x 512 x 31, levels 10-20 with bands 5,
    17 and 28 at 60): every band's level against the oracle."""
    levels = np.linspace(10.0, 20.0, 31)
    levels[[5, 17, 28]] = 60.0
    cube = synth.add_band_awgn(synth.make_hsi(512, 512, 31, seed=7), levels, seed=9)
    got = dn.band_sigma(_dev(cube))
    want = oracle.band_sigma(cube)
    assert np.allclose(got, want, rtol=1e-9, atol=0), (got, want)


def test_band_sigma_in_several_launches(dn):
    """1100 x 1100 x 64: 81 sub-images x 64 bands = 5,184 units, more than one launch takes, so
    the estimates come from two launches; sampled bands against the oracle on each band alone
    (a band's level depends on that band only)."""
    cube = synth.add_band_awgn(synth.make_hsi(1100, 1100, 64, seed=21), np.linspace(5.0, 40.0, 64), seed=22)
    got = dn.band_sigma(_dev(cube))
    for k in (0, 21, 42, 63):
        want = oracle.band_sigma(np.ascontiguousarray(cube[:, :, k:k + 1]))[0]
        assert np.isclose(got[k], want, rtol=1e-9, atol=0), (k, got[k], want)


@pytest.mark.parametrize("levels", [[10, 10, 12, 9, 11, 10, 10, 50], [15.0] * 6])
def test_band_auto_denoise_parity(dn, levels):
    """sigma = AUTO: the cube filtered at the mean band level, severe bands (above twice the mean)
    taken from the cube filtered at the highest level; against the oracle's composition of the
    same two filterings (its band levels, groups and basis)."""
    import paper_2512_23569_amd as ht
    bands, h, w, K, W, s = len(levels), 72, 80, 16, 15, 4
    clean = synth.make_hsi(h, w, bands, 120 + bands)
    noisy = synth.add_band_awgn(clean, np.asarray(levels, dtype=np.float64), 121)
    U, V = lb.learn(noisy, 8, 4)
    ht.htsvd_set_basis(dn.ctx, 8, bands, oracle.to_slices(U), oracle.to_slices(V))
    mean, mx, severe = oracle.band_sigma_rule(oracle.band_sigma(noisy))
    idx, _ = oracle.block_match(oracle.band_guide(noisy), 8, s, W, K)
    mult = np.sqrt(2.0 * np.log(bands * K * 64))
    ref = oracle.filter_groups(noisy, idx, U, V, mean * mult)
    if severe.any():
        hi = oracle.filter_groups(noisy, idx, U, V, mx * mult)
        ref[:, :, severe] = hi[:, :, severe]
    gpu = dn.denoise_bands(_dev(noisy), ht.HTSVD_SIGMA_AUTO, dn.params(1, stride=s, window=W, K=K)).cpu().numpy()
    m = assert_pixel_parity(gpu, ref, clean)
    print("band AUTO levels %s: severe %s" % (levels, severe.nonzero()[0]), m)
    assert severe.any() == (max(levels) > 2 * np.mean(levels))


@pytest.mark.parametrize("bands", [31, 40])
def test_band_unaligned_strided_cube_is_identical(dn, bands):
    """A cube at an odd byte offset with a padded row stride (its rows start at every alignment, so
    the forward kernel's staging copies the chunks outside the cube byte by byte) gives the same
    output as its contiguous copy."""
    h, w = 48, 56
    noisy = synth.add_awgn(synth.make_hsi(h, w, bands, 130 + bands), 20.0, 131 + bands)
    d = _dev(noisy)
    dn.learn_basis(d, stride=4)
    p = dn.params(1, stride=4, window=15, K=8)
    want = dn.denoise_bands(d, 20.0, p)
    stride = w * bands + 5
    flat = torch.zeros(3 + (h - 1) * stride + w * bands, dtype=torch.uint8, device="cuda")
    view = flat.as_strided((h, w, bands), (stride, bands, 1), storage_offset=3)
    view.copy_(d)
    assert view.data_ptr() % 16 == 3 and view.stride(0) == stride
    got = dn.denoise_bands(view, 20.0, p)
    torch.cuda.synchronize()
    assert torch.equal(got, want)


def test_band_full_size_row_band_parity(dn):
    """The benchmark's cube at full size (512 x 512 x 31, AWGN 30, stride 4, window 21, K 16:
    258,064 patches in one pass): rows 248-263 of the GPU output against the oracle's groups
    filter over every group with a member reaching those rows (the only groups that contribute
    to them), with the oracle's learned basis installed on both sides."""
    import paper_2512_23569_amd as ht
    h, w, bands, sigma = 512, 512, 31, 30.0
    clean = synth.make_hsi(h, w, bands, seed=7)
    noisy = synth.add_awgn(clean, sigma, seed=8)
    U, V = lb.learn(noisy, 8, 4)
    ht.htsvd_set_basis(dn.ctx, 8, bands, oracle.to_slices(U), oracle.to_slices(V))
    gpu = dn.denoise_bands(_dev(noisy), sigma, dn.params(1, stride=4, window=21, K=16)).cpu().numpy()
    idx, _ = oracle.block_match(oracle.band_guide(noisy), 8, 4, 21, 16)
    r0, r1 = 248, 264
    rows = idx // w
    sel = np.any((rows <= r1 - 1) & (rows + 7 >= r0), axis=1)
    tau = sigma * np.sqrt(2.0 * np.log(bands * 16 * 64))
    ref = oracle.filter_groups(noisy, idx[sel], U, V, tau)
    m = assert_pixel_parity(gpu[r0:r1], ref[r0:r1], clean[r0:r1])
    print("full-size band rows %d-%d, %d groups:" % (r0, r1 - 1, int(sel.sum())), m)
