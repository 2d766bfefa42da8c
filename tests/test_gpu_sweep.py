"""Parameter sweeps with one grouping pass (the cached patch indices of Sec. III-D-3) on the GPU
(needs an MI355X): group prefixes bit-exact, every sweep output identical to the single call
with the same setting, and one setting against the FP64 oracle."""
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
    d = ht.Denoiser(0, load_network=False)
    yield d
    d.close()


def _dev(img):
    return torch.from_numpy(np.ascontiguousarray(img)).cuda()


@pytest.mark.parametrize("kind,c,s,W", [("clean", 3, 4, 31), ("ties", 3, 3, 15), ("ties", 1, 2, 21),
                                        ("clean", 1, 5, 13)])
def test_smaller_groups_are_prefixes(dn, kind, c, s, W):
    h, w = 70, 83
    img = synth.make_clean(h, w, c, 31) if kind == "clean" else tie_heavy_image(h, w, c, 32)
    d = _dev(img)
    i32, d32 = dn.block_match(d, dn.params(c, stride=s, window=W, K=32))
    for K in (4, 8, 16):
        iK, dK = dn.block_match(d, dn.params(c, stride=s, window=W, K=K))
        torch.cuda.synchronize()
        assert torch.equal(iK, i32[:, :K]) and torch.equal(dK, d32[:, :K]), K


SETTINGS = [(25.0, 16), (40.0, 32), (25.0, 32), (60.0, 8), (10.0, 4), (40.0, 16)]


@pytest.mark.parametrize("c,h,w,W", [(3, 200, 160, 31), (1, 131, 97, 21)])
def test_sweep_equals_single_calls(dn, c, h, w, W):
    clean = synth.make_clean(h, w, c, 33)
    noisy = synth.add_awgn(clean, 35.0, 34)
    d = _dev(noisy)
    p = dn.params(c, stride=3, window=W, K=32)
    outs = dn.denoise_sweep(d, SETTINGS, p)
    for (sigma, K), o in zip(SETTINGS, outs):
        single = dn.denoise(d, sigma, p.replace(K=K))
        torch.cuda.synchronize()
        assert torch.equal(o, single), (sigma, K)


def test_sweep_with_smaller_max_group_and_tau_mult(dn):
    noisy = synth.add_awgn(synth.make_clean(96, 120, 3, 35), 20.0, 36)
    d = _dev(noisy)
    p = dn.params(3, stride=4, window=21, K=16, tau_mult=2.5)
    settings = [(20.0, 8), (20.0, 16), (30.0, 4)]
    outs = dn.denoise_sweep(d, settings, p)
    for (sigma, K), o in zip(settings, outs):
        assert torch.equal(o, dn.denoise(d, sigma, p.replace(K=K))), (sigma, K)


def test_sweep_setting_against_oracle(dn, basis3):
    """A K = 16 setting of a K = 32 sweep: the pixel parity bar against the oracle's own
    16-member grouping and filter."""
    clean = synth.make_clean(128, 144, 3, 37)
    noisy = synth.add_awgn(clean, 30.0, 38)
    U, V = basis3
    d = _dev(noisy)
    p = dn.params(3, stride=4, window=21, K=32)
    out16, out32 = dn.denoise_sweep(d, [(30.0, 16), (30.0, 32)], p)
    for K, o in ((16, out16), (32, out32)):
        ref = oracle.denoise(noisy, U, V, 30.0 * oracle.tau_multiplier(3, K), s=4, W=21, K=K)
        m = assert_pixel_parity(o.cpu().numpy(), ref, clean)
        print("sweep K=%d" % K, m)


def test_sweep_errors_are_reported(dn):
    import paper_2512_23569_amd as ht
    d = _dev(synth.make_clean(48, 48, 3, 39))
    p = dn.params(3, stride=4, window=21, K=16)
    for bad in ([(20.0, 32)], [(0.0, 16)], [(20.0, 12)], []):
        with pytest.raises(ht.HtsvdError):
            dn.denoise_sweep(d, bad, p)
    with pytest.raises(ht.HtsvdError):
        dn.denoise_sweep(d, [(20.0, 16)], p.replace(adaptive=1))
