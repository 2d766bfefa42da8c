"""GPU path vs the FP64 oracle through the C ABI (needs an MI355X)."""
import numpy as np
import pytest

import oracle
import synth
from helpers import assert_pixel_parity, tie_heavy_image

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dn():
    import paper_2512_23569_amd as ht
    assert torch.cuda.is_available(), "GPU tests need a device"
    d = ht.Denoiser(0)
    yield d
    d.close()


def _dev(img):
    return torch.from_numpy(np.ascontiguousarray(img)).cuda()


def _gpu_groups(dn, img, **kw):
    c = 3 if img.ndim == 3 else 1
    p = dn.params(c, **kw)
    idx, dist = dn.block_match(_dev(img), p)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), dist.cpu().numpy()


def _check_groups(dn, img, s, W, K):
    gi, gd = _gpu_groups(dn, img, stride=s, window=W, K=K)
    oi, od = oracle.block_match(img, 8, s, W, K)
    bad = np.nonzero(np.any(gi != oi, axis=1) | np.any(gd != od, axis=1))[0]
    assert bad.size == 0, "first mismatching reference %d: gpu %s / %s oracle %s / %s" % (
        bad[0], gi[bad[0]], gd[bad[0]], oi[bad[0]], od[bad[0]])


def test_groups_bitexact_gray256(dn):
    clean, noisy, _ = synth.make_cfg("gray256_awgn25")
    _check_groups(dn, noisy, 4, 21, 16)


def test_groups_bitexact_rgb512(dn):
    clean, noisy, _ = synth.make_cfg("rgb512_awgn50")
    _check_groups(dn, noisy, 4, 31, 32)


@pytest.mark.parametrize("h,w,c,s,W,K,seed", [
    (37, 45, 1, 3, 9, 8, 0), (40, 29, 3, 1, 7, 16, 1), (64, 70, 3, 5, 31, 32, 2),
    (9, 11, 1, 1, 3, 4, 3),
    (50, 33, 3, 11, 31, 4, 4), (100, 37, 1, 2, 15, 32, 5), (23, 91, 3, 4, 21, 16, 6),
])
def test_groups_bitexact_ragged_and_ties(dn, h, w, c, s, W, K, seed):
    _check_groups(dn, tie_heavy_image(h, w, c, seed), s, W, K)
    clean = synth.make_clean(h, w, c, seed)
    _check_groups(dn, synth.add_awgn(clean, 30.0, seed + 7), s, W, K)


def test_groups_flat_image(dn):
    for c in (1, 3):
        img = np.full((30, 34, 3) if c == 3 else (30, 34), 128, np.uint8)
        _check_groups(dn, img, 3, 11, 16)


def _tau_dev(tau):
    return torch.from_numpy(np.ascontiguousarray(tau, dtype=np.float64)).cuda()


def _denoise_tau(dn, img, tau_ref, **kw):
    c = 3 if img.ndim == 3 else 1
    p = dn.params(c, **kw)
    out = dn.denoise_tau(_dev(img), _tau_dev(tau_ref), p)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_denoise_parity_gray256(dn, basis1):
    clean, noisy, _ = synth.make_cfg("gray256_awgn25")
    U, V = basis1
    ny, nx = oracle.n_refs(256, 256, 8, 4)
    tau = np.full(ny * nx, 25.0 * oracle.tau_multiplier(1, 16))
    ref = oracle.denoise(noisy, U, V, tau, s=4, W=21, K=16)
    gpu = _denoise_tau(dn, noisy, tau, stride=4, window=21, K=16)
    m = assert_pixel_parity(gpu, ref, clean)
    print("gray256", m, "guard", dn.guard_count())


def test_denoise_parity_rgb512(dn, basis3):
    clean, noisy, _ = synth.make_cfg("rgb512_awgn50")
    U, V = basis3
    ny, nx = oracle.n_refs(512, 512, 8, 4)
    tau = np.full(ny * nx, 50.0 * oracle.tau_multiplier(3, 32))
    ref = oracle.denoise(noisy, U, V, tau, s=4, W=31, K=32)
    gpu = _denoise_tau(dn, noisy, tau, stride=4, window=31, K=32)
    m = assert_pixel_parity(gpu, ref, clean)
    print("rgb512", m, "guard", dn.guard_count())


def test_denoise_known_sigma_equals_tau_path(dn):
    clean, noisy, _ = synth.make_cfg("gray256_awgn25", h=96, w=80)
    p = dn.params(1, stride=4, window=21, K=16)
    a = dn.denoise(_dev(noisy), 25.0, p).cpu().numpy()
    ny, nx = oracle.n_refs(96, 80, 8, 4)
    b = _denoise_tau(dn, noisy, np.full(ny * nx, 25.0 * oracle.tau_multiplier(1, 16)), stride=4, window=21, K=16)
    assert np.max(np.abs(a - b)) < 1e-3


@pytest.mark.parametrize("c,K,s,W", [(1, 4, 1, 5), (3, 8, 3, 9), (3, 16, 2, 15), (1, 32, 5, 31)])
def test_denoise_parity_small_variants(dn, basis1, basis3, c, K, s, W):
    h, w = 41, 53
    clean = synth.make_clean(h, w, c, 40 + K)
    noisy = synth.add_awgn(clean, 20.0, 41 + K)
    U, V = basis3 if c == 3 else basis1
    ny, nx = oracle.n_refs(h, w, 8, s)
    tau = np.random.default_rng(K).uniform(30, 120, ny * nx)  # per-reference thresholds
    ref = oracle.denoise(noisy, U, V, tau, s=s, W=W, K=K)
    gpu = _denoise_tau(dn, noisy, tau, stride=s, window=W, K=K)
    assert_pixel_parity(gpu, ref, clean)


def test_perfect_reconstruction_and_total_kill(dn):
    for c in (1, 3):
        clean = synth.make_clean(48, 56, c, 77)
        noisy = synth.add_awgn(clean, 15.0, 78)
        ny, nx = oracle.n_refs(48, 56, 8, 3)
        out0 = _denoise_tau(dn, noisy, np.zeros(ny * nx), stride=3, window=9, K=8)
        assert np.max(np.abs(out0 - noisy)) < 1e-3
        outinf = _denoise_tau(dn, noisy, np.full(ny * nx, np.inf), stride=3, window=9, K=8)
        assert np.max(np.abs(outinf)) == 0.0


def test_errors_are_reported(dn):
    import paper_2512_23569_amd as ht
    img = _dev(np.zeros((32, 32), np.uint8))
    with pytest.raises(ht.HtsvdError) as e:
        dn.denoise(img, 10.0, dn.params(1, window=20))
    assert e.value.status == ht.HTSVD_EINVAL
    with pytest.raises(ht.HtsvdError) as e:
        dn.denoise(img, 10.0, dn.params(1, K=12))
    assert e.value.status == ht.HTSVD_ENOTSUP
    with pytest.raises(ht.HtsvdError) as e:
        dn.denoise(_dev(np.zeros((9, 9), np.uint8)), 10.0, dn.params(1, window=3, K=8))
    assert e.value.status == ht.HTSVD_ESHAPE
