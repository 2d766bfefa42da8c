"""Noise estimation and the Eq. 23 vote on the GPU vs the oracle (needs an MI355X)."""
import numpy as np
import pytest

import oracle
import synth
from helpers import assert_pixel_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dn():
    import paper_2512_23569_amd as ht
    assert torch.cuda.is_available(), "GPU tests need a device"
    d = ht.Denoiser(0)
    yield d
    d.close()


def _gpu_sigma(dn, img, sigma, **kw):
    import paper_2512_23569_amd as ht
    c = 3 if img.ndim == 3 else 1
    p = dn.params(c, **kw)
    h, w = img.shape[:2]
    nt = ((h + 127) // 128) * ((w + 127) // 128)
    se = torch.zeros(nt, dtype=torch.float64, device="cuda")
    sh = torch.zeros(nt, dtype=torch.float64, device="cuda")
    vo = torch.zeros(nt, dtype=torch.int32, device="cuda")
    d_in = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    ht.htsvd_estimate_sigma(dn.ctx, d_in, h, w, c, d_in.stride(0), sigma, p, se, sh, vo)
    torch.cuda.synchronize()
    return se.cpu().numpy(), sh.cpu().numpy(), vo.cpu().numpy()


@pytest.mark.parametrize("h,w,c,sigma,seed", [(256, 256, 1, 25.0, 1), (300, 430, 3, 40.0, 2), (130, 70, 3, 10.0, 3)])
def test_sigma_est_matches_oracle(dn, h, w, c, sigma, seed):
    clean = synth.make_clean(h, w, c, seed)
    noisy = synth.add_awgn(clean, sigma, seed + 1)
    se, _, _ = _gpu_sigma(dn, noisy, -1.0)
    ref = oracle.sigma_est_tiles(noisy)
    assert np.allclose(se, ref, rtol=1e-9, atol=0), (se, ref)


def test_sigma_est_flat_awgn(dn):
    noisy = synth.add_awgn(np.full((256, 384, 3), 120, np.uint8), 20.0, 9)
    se, _, _ = _gpu_sigma(dn, noisy, -1.0)
    assert np.all(np.abs(se / 20.0 - 1) < 0.03), se


@pytest.mark.parametrize("c,K,s,W,sigma", [(3, 32, 4, 31, 50.0), (1, 16, 4, 21, 25.0), (3, 16, 3, 15, 10.0)])
def test_votes_match_oracle(dn, c, K, s, W, sigma):
    h, w = 300, 270
    clean = synth.make_clean(h, w, c, 30 + K)
    noisy = synth.add_awgn(clean, sigma, 31 + K)
    se, sh, vo = _gpu_sigma(dn, noisy, sigma, stride=s, window=W, K=K, adaptive=1)
    idx, _ = oracle.block_match(noisy, 8, s, W, K)
    nt = se.size
    ref_hat, ref_votes, _, _ = oracle.sigma_hat_tiles(noisy, idx, np.full(nt, sigma), 8, s, return_votes=True)
    assert np.array_equal(vo, ref_votes), (vo, ref_votes)
    assert np.array_equal(sh, ref_hat)


def test_adaptive_auto_denoise_parity(dn, basis3):
    clean, noisy, _ = synth.make_cfg("rgb512_awgn50", h=256, w=320)
    p = dn.params(3, stride=4, window=31, K=32, adaptive=1)
    gpu = dn.denoise(torch.from_numpy(noisy).cuda(), -1.0, p).cpu().numpy()
    U, V = basis3
    idx, _ = oracle.block_match(noisy, 8, 4, 31, 32)
    sig = oracle.sigma_hat_tiles(noisy, idx, oracle.sigma_est_tiles(noisy), 8, 4)
    tau = oracle.tau_per_ref(sig, 256, 320, 8, 4, 3, 32)
    ref = oracle.denoise(noisy, U, V, tau, s=4, W=31, K=32)
    m = assert_pixel_parity(gpu, ref, clean)
    print("adaptive auto", m, sig)


def test_adaptive_known_sigma_denoise_parity(dn, basis3):
    clean, noisy, _ = synth.make_cfg("rgb512_awgn50")
    p = dn.params(3, stride=4, window=31, K=32, adaptive=1)
    gpu = dn.denoise(torch.from_numpy(noisy).cuda(), 50.0, p).cpu().numpy()
    U, V = basis3
    idx, _ = oracle.block_match(noisy, 8, 4, 31, 32)
    sig = oracle.sigma_hat_tiles(noisy, idx, np.full(16, 50.0), 8, 4)
    tau = oracle.tau_per_ref(sig, 512, 512, 8, 4, 3, 32)
    ref = oracle.denoise(noisy, U, V, tau, s=4, W=31, K=32)
    m = assert_pixel_parity(gpu, ref, clean)
    print("adaptive known", m, sig)
