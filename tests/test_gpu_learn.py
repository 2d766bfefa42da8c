"""Basis learned from the image itself (Sec. III-B, Eq. 10-11) on the GPU vs the FP64 oracle
(needs an MI355X): the Gram sums bit-exact, the learned pair to 1e-9, the denoised image to
the pixel parity bar."""
import numpy as np
import pytest

import oracle
import synth
from helpers import assert_pixel_parity, tie_heavy_image
from oracle import learn_basis as lb

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# The Gram sums are exact integers on both sides, so the only differences in the pair come from
# the two eigensolvers (LAPACK's and the library's Jacobi) and the FP64 DFT: a few 1e-13 on these
# inputs, whose eigenvalues are well separated.
BASIS_TOL = 1e-9


@pytest.fixture(scope="module")
def dn():
    import paper_2512_23569_amd as ht
    assert torch.cuda.is_available(), "GPU tests need a device"
    d = ht.Denoiser(0, load_network=False)
    yield d
    d.close()


def _dev(img):
    return torch.from_numpy(np.ascontiguousarray(img)).cuda()


def _gram(dn, img, s):
    G = dn.basis_gram(_dev(img), stride=s)
    torch.cuda.synchronize()
    return G.cpu().numpy()


@pytest.mark.parametrize("h,w,c,s,seed", [(8, 8, 1, 4, 1), (8, 8, 3, 1, 2), (9, 40, 3, 7, 3), (41, 53, 1, 5, 4),
                                          (77, 93, 3, 3, 5), (130, 257, 3, 1, 6), (256, 256, 1, 4, 7),
                                          (300, 517, 3, 4, 8), (64, 64, 3, 9, 9)])
def test_gram_sums_bit_exact(dn, h, w, c, s, seed):
    img = synth.make_clean(h, w, c, seed)
    want = lb.channel_gram(img, 8, s)
    got = _gram(dn, img, s)
    assert got.dtype == np.int64 and np.array_equal(got, want), np.argwhere(got != want)[:5]


def test_gram_sums_tie_heavy_and_padded_rows(dn):
    img = tie_heavy_image(70, 90, 3, 11)
    big = np.zeros((70, 100, 3), dtype=np.uint8)
    big[:, :90] = img
    t = _dev(big)[:, :90]   # rows 300 bytes apart, 270 used
    G = dn.basis_gram(t, stride=3)
    torch.cuda.synchronize()
    assert np.array_equal(G.cpu().numpy(), lb.channel_gram(img, 8, 3))


def test_gram_sums_saturated_image_at_full_size(dn):
    """All pixels 255 at 12 MP and stride 1 (the largest sums): every entry is
    (number of patches) * 8 * 255^2."""
    h, w = 3000, 4000
    img = torch.full((h, w, 3), 255, dtype=torch.uint8, device="cuda")
    G = dn.basis_gram(img, stride=1)
    torch.cuda.synchronize()
    n = oracle.n_refs(h, w, 8, 1)
    want = n[0] * n[1] * 8 * 255 * 255
    assert np.all(G.cpu().numpy() == want)


def test_gram_sums_full_size_workload(dn):
    """The 12 MP benchmark image (Poisson-Gaussian noise) at stride 4, against the oracle's sums."""
    _, noisy, _ = synth.make_cfg("rgb12mp_pg")
    got = _gram(dn, noisy, 4)
    assert np.array_equal(got, lb.channel_gram(noisy, 8, 4))


@pytest.mark.parametrize("name,c,s", [("rgb512", 3, 4), ("gray256", 1, 4), ("rgb_noisy", 3, 4), ("ragged", 3, 3),
                                      ("gray_ragged", 1, 2)])
def test_learned_basis_matches_oracle(dn, name, c, s):
    if name == "rgb512":
        img = synth.make_clean(512, 512, 3, seed=0)
    elif name == "gray256":
        img = synth.make_clean(256, 256, 1, seed=1)
    elif name == "rgb_noisy":
        img = synth.add_awgn(synth.make_clean(256, 192, 3, seed=3), 25.0, 5)
    elif name == "ragged":
        img = synth.make_clean(77, 93, 3, seed=7)
    else:
        img = synth.add_awgn(synth.make_clean(61, 45, 1, seed=8), 10.0, 9)
    Ug, Vg = dn.learn_basis(_dev(img), stride=s)
    Uo, Vo = lb.learn(img, 8, s)
    du = np.abs(Ug - oracle.to_slices(Uo)).max()
    dv = np.abs(Vg - oracle.to_slices(Vo)).max()
    print(name, "max |dU| %.3g |dV| %.3g" % (du, dv))
    assert du <= BASIS_TOL and dv <= BASIS_TOL


def test_learned_basis_of_a_flat_image_is_valid(dn):
    """A constant image with three different channel values: every slice covariance is a
    positive multiple of the all-ones matrix, so each slice's first vector is 1/sqrt(8) in every
    entry (the real tensor: 1/sqrt(8) on slice 0 of the first column, 0 on the others) and the
    other vectors are not unique: checked for orthonormality only."""
    img = np.empty((24, 32, 3), dtype=np.uint8)
    img[:] = (77, 140, 20)
    Ug, Vg = dn.learn_basis(_dev(img), stride=4)
    for T in (Ug, Vg):
        assert np.allclose(T[0, :, 0], 1 / np.sqrt(8), atol=1e-12)
        assert np.allclose(T[1:, :, 0], 0.0, atol=1e-12)
        Th = np.fft.fft(T, axis=0)
        for f in range(3):
            assert np.allclose(Th[f][:, 0], 1 / np.sqrt(8), atol=1e-12)
            assert np.allclose(Th[f].conj().T @ Th[f], np.eye(8), atol=1e-12)


def test_denoise_with_learned_basis_parity(dn):
    """Learn the pair from the noisy image itself, then denoise with it: GPU learning + GPU
    filter against oracle learning + oracle filter."""
    clean = synth.make_clean(192, 160, 3, seed=12)
    noisy = synth.add_awgn(clean, 30.0, 13)
    dn.learn_basis(_dev(noisy), stride=4)
    U, V = lb.learn(noisy, 8, 4)
    ny, nx = oracle.n_refs(192, 160, 8, 4)
    tau = np.full(ny * nx, 30.0 * oracle.tau_multiplier(3, 16))
    ref = oracle.denoise(noisy, U, V, tau, s=4, W=21, K=16)
    p = dn.params(3, stride=4, window=21, K=16)
    gpu = dn.denoise_tau(_dev(noisy), torch.from_numpy(tau).cuda(), p).cpu().numpy()
    m = assert_pixel_parity(gpu, ref, clean)
    print("learned-basis denoise", m)


def test_learning_errors_are_reported(dn):
    import paper_2512_23569_amd as ht
    img = _dev(synth.make_clean(32, 32, 3, seed=1))
    out = torch.empty((2, 3, 3, 8, 8), dtype=torch.int64, device="cuda")
    with pytest.raises(ht.HtsvdError):
        ht.htsvd_basis_gram(dn.ctx, img, 32, 32, 3, 96, 8, 0, out)       # stride 0
    with pytest.raises(ht.HtsvdError):
        ht.htsvd_basis_gram(dn.ctx, img, 32, 32, 3, 96, 16, 4, out)      # ps 16
    with pytest.raises(ht.HtsvdError):
        ht.htsvd_basis_gram(dn.ctx, img, 32, 32, 3, 95, 8, 4, out)       # in_stride < w*c
    with pytest.raises(ht.HtsvdError):
        ht.htsvd_learn_basis(dn.ctx, img, 7, 32, 3, 96, 8, 4)            # smaller than a patch
    with pytest.raises(ht.HtsvdError):
        ht.htsvd_learn_basis(dn.ctx, img, 32, 32, 65, 96, 8, 4)          # 65 channels (2 .. 64 are bands)
