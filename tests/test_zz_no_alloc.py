"""htsvd_denoise_noalloc, the entry point that allocates nothing (needs an MI355X): its scratch
lives in the library's fixed per-GPU array.  It runs the kernels of htsvd_denoise with the
same tiling, so its output is compared with htsvd_denoise's on the same input (the pixel parity
bar, and the bound between GPU runs of the fixed-point aggregation), on two calls in a row, the
second with a smaller image, for a known and an estimated noise level; and an image too large
for the array is refused before anything runs."""
import ctypes

import numpy as np
import pytest

import synth
from helpers import assert_pixel_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RUN_TOL = 2e-3


@pytest.fixture(scope="module")
def dn():
    import paper_2512_23569_amd as ht
    assert torch.cuda.is_available(), "GPU tests need a device"
    d = ht.Denoiser(0, load_network=False)
    yield d
    d.close()


def _call_noalloc(dn, x, sigma, p, out):
    """Through the C entry point itself (ctypes), with explicit strides."""
    import paper_2512_23569_amd as ht
    h, w, c = x.shape
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = ht.lib().htsvd_denoise_noalloc(dn.ctx, ctypes.c_void_p(x.data_ptr()), h, w, c, x.stride(0),
                                        ctypes.c_float(sigma), ctypes.byref(p), ctypes.c_void_p(out.data_ptr()),
                                        out.stride(0), st)
    return rc


@pytest.mark.parametrize("sigma,adaptive", [(30.0, 0), (-1.0, 1)])
def test_noalloc_matches_denoise_on_two_calls(dn, sigma, adaptive):
    import paper_2512_23569_amd as ht
    p = dn.params(3, stride=4, window=31, K=32, adaptive=adaptive, estimator=0)
    for (h, w), seed in (((384, 512), 11), ((200, 264), 12)):     # the second call is smaller
        clean = synth.make_clean(h, w, 3, seed)
        noisy = synth.add_awgn(clean, 30.0, seed + 100)
        x = torch.from_numpy(noisy).cuda()
        out = torch.full((h, w, 3), -5.0, dtype=torch.float32, device="cuda")
        assert _call_noalloc(dn, x, sigma, p, out) == ht.HTSVD_OK, ht.htsvd_last_error()
        got = out.cpu().numpy()
        want = dn.denoise(x, sigma, p).cpu().numpy()
        assert np.max(np.abs(got - want)) <= RUN_TOL, ((h, w), float(np.max(np.abs(got - want))))
        assert_pixel_parity(got, want, clean)


def test_noalloc_refuses_what_it_cannot_hold(dn):
    import paper_2512_23569_amd as ht
    h, w = 2048, 2048
    x = torch.zeros((h, w, 3), dtype=torch.uint8, device="cuda")
    out = torch.zeros((h, w, 3), dtype=torch.float32, device="cuda")
    p = dn.params(3, stride=4, window=31, K=32)
    assert _call_noalloc(dn, x, 25.0, p, out) == ht.HTSVD_ENOMEM
    assert "scratch" in ht.htsvd_last_error()
    small = x[:64, :64].contiguous()
    assert _call_noalloc(dn, small, -1.0, p.replace(estimator=1), out) == ht.HTSVD_ENOTSUP   # learned map
    assert _call_noalloc(dn, small, 25.0, p.replace(ra=1), out) == ht.HTSVD_ENOTSUP          # RA network
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0      # nothing was written
