"""The batched persistent launch (one work-queue launch per stage for a whole batch, optionally
replayed from a hipGraph) vs the FP64 oracle and vs the one-image entry points (needs an MI355X).

Filtering accumulates the reconstructed patches in LDS as int32 fixed point (units of 2^-FS,
9 <= FS <= 12 chosen per tiling so that no sum can overflow), so two runs
with the same tiling give identical results, and runs with different tilings differ by at most
the rounding of one fixed-point unit per run (2 * 2^-(FS+1) <= 2^-9 on the 0..255 scale).  Comparisons
between GPU runs allow RUN_TOL; comparisons with the oracle use the pixel parity bar."""
import numpy as np
import pytest

import oracle
import synth
from helpers import assert_pixel_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RUN_TOL = 2e-3


@pytest.fixture(scope="module")
def dn():
    import paper_2512_23569_amd as ht
    assert torch.cuda.is_available(), "GPU tests need a device"
    d = ht.Denoiser(0)
    yield d
    d.close()


def _dev(img):
    return torch.from_numpy(np.ascontiguousarray(img)).cuda()


def _mixed_batch(c, seed):
    shapes = [(64, 72), (41, 53), (96, 40), (17, 130), (33, 33), (120, 88)]
    sig = [10.0, 25.0, 50.0, 15.0, 40.0, 30.0]
    cl, nz = [], []
    for i, (h, w) in enumerate(shapes):
        clean = synth.make_clean(h, w, c, seed + i)
        cl.append(clean)
        nz.append(synth.add_awgn(clean, sig[i], seed + 100 + i))
    return cl, nz, sig


@pytest.mark.parametrize("c", [3, 1])
def test_batch_matches_oracle_per_image(dn, basis1, basis3, c):
    """Every image of a mixed-size, mixed-K batch equals the oracle with that image's tau."""
    cl, nz, sig = _mixed_batch(c, 10 * c)
    Ks = [16, 32, 16, 32, 8, 16]
    s, W = 3, 15
    p = dn.params(c, stride=s, window=W)
    outs = dn.denoise_batch([_dev(x) for x in nz], sig, p, Ks=Ks)
    torch.cuda.synchronize()
    U, V = basis3 if c == 3 else basis1
    for i, x in enumerate(nz):
        h, w = x.shape[:2]
        ny, nx = oracle.n_refs(h, w, 8, s)
        tau = np.full(ny * nx, sig[i] * oracle.tau_multiplier(c, Ks[i]))
        ref = oracle.denoise(x, U, V, tau, s=s, W=W, K=Ks[i])
        assert_pixel_parity(outs[i].cpu().numpy(), ref, cl[i])


def test_batch_equals_single_image_calls(dn):
    cl, nz, sig = _mixed_batch(3, 5)
    p = dn.params(3, stride=4, window=21, K=32)
    outs = dn.denoise_batch([_dev(x) for x in nz], sig, p, use_graph=False, blocks_per_cu=2)
    for i, x in enumerate(nz):
        one = dn.denoise(_dev(x), sig[i], p)
        assert torch.max(torch.abs(outs[i] - one)).item() <= RUN_TOL


def test_graph_replays_match_eager(dn):
    """The captured graph replayed several times, with eager work and synchronisations in
    between, gives the eager result each time, and follows new input contents."""
    cl, nz, sig = _mixed_batch(3, 7)
    p = dn.params(3, stride=3, window=15, K=16)
    ins = [_dev(x) for x in nz]
    eager = [o.clone() for o in dn.denoise_batch(ins, sig, p, use_graph=False)]
    outs = [torch.empty(x.shape, dtype=torch.float32, device="cuda") for x in ins]
    for rep in range(4):
        for o in outs:
            o.fill_(-7.0)
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work between replays
        dn.denoise_batch(ins, sig, p, outs=outs, use_graph=True)
        torch.cuda.synchronize()
        assert np.isfinite(junk.item())
        for e, o in zip(eager, outs):
            assert torch.max(torch.abs(e - o)).item() <= RUN_TOL, rep
    # same pointers, new contents: the replay recomputes
    new = synth.add_awgn(cl[0], sig[0], 999)
    ins[0].copy_(_dev(new))
    dn.denoise_batch(ins, sig, p, outs=outs, use_graph=True)
    one = dn.denoise(ins[0], sig[0], p)
    assert torch.max(torch.abs(outs[0] - one)).item() <= RUN_TOL


def test_batch_estimated_sigma_matches_single(dn):
    """Images with an estimated noise level (plain estimator with the vote, and the learned
    map when a network is loaded) give the one-image results inside a batch."""
    clean, noisy, _ = synth.make_cfg("rgb512_awgn50", h=200, w=260)
    c2 = synth.make_clean(150, 129, 3, 3)
    n2 = synth.add_awgn(c2, 20.0, 4)
    ins = [_dev(noisy), _dev(n2)]
    for est in (0, 1):
        p = dn.params(3, stride=4, window=21, K=16, adaptive=1, estimator=est)
        outs = dn.denoise_batch(ins, [-1.0, 20.0], p)
        for i, x in enumerate(ins):
            one = dn.denoise(x, [-1.0, 20.0][i], p)
            assert torch.max(torch.abs(outs[i] - one)).item() <= RUN_TOL, (est, i)


def test_batch_errors(dn):
    import paper_2512_23569_amd as ht
    a = _dev(np.zeros((32, 32, 3), np.uint8))
    b = _dev(np.zeros((32, 32), np.uint8))
    with pytest.raises(ht.HtsvdError) as e:
        dn.denoise_batch([a, b], [10.0, 10.0], dn.params(3))
    assert e.value.status == ht.HTSVD_ENOTSUP
    with pytest.raises(ht.HtsvdError) as e:
        dn.denoise_batch([a], [10.0], dn.params(3), Ks=[12])
    assert e.value.status == ht.HTSVD_ENOTSUP
    with pytest.raises(ht.HtsvdError) as e:
        dn.denoise_batch([a], [0.0], dn.params(3))
    assert e.value.status == ht.HTSVD_EINVAL


def test_auto_group_size_follows_the_sigma_cutoff(dn):
    """HTSVD_K_AUTO: images whose mean noise level is below the cutoff are filtered with the first
    16 members of their 32-member groups, the others with 32; each output equals the one-image
    call with that K (known sigma, and the plain estimate without the vote)."""
    import paper_2512_23569_amd as ht
    cl, nz, sig = _mixed_batch(3, 21)
    ins = [_dev(x) for x in nz]
    cutoff = 20.0   # 5 units from the nearest level of the batch (15 and 25)
    for adaptive_sigma in (False, True):
        sigmas = [-1.0] * len(ins) if adaptive_sigma else sig
        p = dn.params(3, stride=4, window=21, adaptive=0, estimator=0)
        outs = dn.denoise_batch(ins, sigmas, p, Ks=[ht.HTSVD_K_AUTO] * len(ins), k_sigma_cutoff=cutoff)
        for i, x in enumerate(ins):
            K = 16 if sig[i] < cutoff else 32
            one = dn.denoise(x, sigmas[i], p.replace(K=K))
            assert torch.max(torch.abs(outs[i] - one)).item() <= RUN_TOL, (adaptive_sigma, i, sig[i])


def test_auto_group_size_in_graph_replays(dn):
    import paper_2512_23569_amd as ht
    cl, nz, sig = _mixed_batch(3, 31)
    ins = [_dev(x) for x in nz]
    p = dn.params(3, stride=3, window=15, adaptive=1, estimator=1)
    Ks = [ht.HTSVD_K_AUTO, 32, ht.HTSVD_K_AUTO, 16, ht.HTSVD_K_AUTO, ht.HTSVD_K_AUTO]
    eager = [o.clone() for o in dn.denoise_batch(ins, [-1.0] * 6, p, Ks=Ks, use_graph=False, k_sigma_cutoff=30.0)]
    for rep in range(3):
        outs = dn.denoise_batch(ins, [-1.0] * 6, p, Ks=Ks, use_graph=True, k_sigma_cutoff=30.0,
                                tile_side=4)
        torch.cuda.synchronize()
        for e, o in zip(eager, outs):
            assert torch.max(torch.abs(e - o)).item() <= RUN_TOL, rep


def test_learned_images_of_one_size_share_a_network_run(dn):
    """Learned images are grouped by size and the network runs once per size class (input
    layer through a pointer table, maps contiguous per class): three images of one size, each in
    its own buffer with its own row padding, and one of another size give the one-image results."""
    shapes = [(96, 80), (96, 80), (70, 130), (96, 80)]
    sig = [12.0, 35.0, 20.0, 60.0]
    ins, outs = [], []
    for i, (h, w) in enumerate(shapes):
        clean = synth.make_clean(h, w, 3, 500 + i)
        noisy = synth.add_awgn(clean, sig[i], 600 + i)
        pad = 3 * i   # different row strides within the class
        buf = torch.zeros((h, w * 3 + pad), dtype=torch.uint8, device="cuda")
        buf[:, : w * 3] = _dev(noisy).reshape(h, w * 3)
        ins.append(buf[:, : w * 3].reshape(h, w, 3) if pad == 0 else buf.as_strided((h, w, 3), (w * 3 + pad, 3, 1)))
    for est in (1, 0):
        p = dn.params(3, stride=3, window=15, K=16, adaptive=1, estimator=est)
        outs = dn.denoise_batch(ins, [-1.0] * len(ins), p, use_graph=True)
        torch.cuda.synchronize()
        for i, x in enumerate(ins):
            one = dn.denoise(x, -1.0, p)
            assert torch.max(torch.abs(outs[i] - one)).item() <= RUN_TOL, (est, i)
