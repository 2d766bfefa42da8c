"""Pins of the oracle's learned-noise-map rule (Sec. III-E-1, Eq. 22-23): how a per-8x8-block
log(sigma) map becomes per-reference thresholds.  The rule (the library's reading): a
sub-image keeps the map when its mean learned sigma lies within a factor 1.5 of the plain
estimate; the Eq. 23 vote scales the tile's level; a reference takes the effective sigma of the
block holding its top-left pixel.

Each pin takes an independent route: exact binary boundary values for the judge, pixel
membership for the blocks of a sub-image, an explicit search for the block holding a pixel,
hand-computed means, and the reduction to the plain rule when every tile rejects the map."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import estimator as est


def test_judge_boundary_is_inclusive_on_both_sides():
    # mean 3, plain 2: ratio exactly 1.5 (1.5 * 2 == 3 exactly) -> kept
    assert est.judge_tile_sigma([3.0] * 4, 2.0) == (3.0, False)
    sp = math.nextafter(2.0, 0.0)            # ratio just above 1.5 -> rejected
    assert est.judge_tile_sigma([3.0] * 4, sp) == (sp, True)
    # mean 2, plain 3: ratio exactly 1/1.5 -> kept; plain a hair larger -> rejected
    assert est.judge_tile_sigma([2.0] * 4, 3.0) == (2.0, False)
    sp = math.nextafter(3.0, 10.0)
    assert est.judge_tile_sigma([2.0] * 4, sp) == (sp, True)
    # the mean, not a single block, is judged: 1 and 5 average to 3
    assert est.judge_tile_sigma([1.0, 5.0], 2.0) == (3.0, False)
    # non-finite or non-positive values fall back to the plain estimate
    assert est.judge_tile_sigma([np.inf, 1.0], 2.0) == (2.0, True)
    assert est.judge_tile_sigma([0.0, 0.0], 2.0) == (2.0, True)
    assert est.judge_tile_sigma([3.0], 0.0) == (0.0, True)


@pytest.mark.parametrize("h,w", [(200, 300), (128, 256), (129, 8), (8, 8), (257, 131), (384, 130)])
def test_blocks_of_a_tile_by_pixel_membership(h, w):
    nty, ntx = est.tile_grid(h, w)
    seen = np.zeros((-(-h // 8), -(-w // 8)), dtype=int)
    for t in range(nty * ntx):
        ty, tx = divmod(t, ntx)
        # blocks containing any pixel of the tile, by brute force over its pixels
        want = {(y // 8, x // 8) for y in range(ty * 128, min(h, ty * 128 + 128))
                for x in range(tx * 128, min(w, tx * 128 + 128))}
        by0, by1, bx0, bx1 = est.blocks_of_tile(t, h, w)
        got = {(by, bx) for by in range(by0, by1) for bx in range(bx0, bx1)}
        assert got == want
        for by, bx in got:
            seen[by, bx] += 1
    assert np.all(seen == 1)   # every block in exactly one tile


def test_learned_judge_hand_means():
    h, w = 200, 300                      # tiles 2 x 3, the last row and column partial
    hb, wb = 25, 38
    z = np.zeros((hb, wb))
    vals = [10.0, 20.0, 30.0, 40.0, 50.0, 60.0]
    for t, v in enumerate(vals):
        by0, by1, bx0, bx1 = est.blocks_of_tile(t, h, w)
        z[by0:by1, bx0:bx1] = np.log(v)
    # the partial corner tile: blocks rows 16..24, cols 32..37 (9 x 6 = 54 blocks); half of
    # them at sigma 40, half at 80 -> mean 60
    z[16:25, 32:35] = np.log(40.0)
    z[16:25, 35:38] = np.log(80.0)
    sp = np.array([10.0 * 1.4, 20.0 / 1.4, 30.0 * 1.6, 40.0 / 1.6, 50.0, 60.0 * 1.45])
    se, up = est.learned_judge(z, sp, h, w)
    assert list(up) == [False, False, True, True, False, False]
    want = np.array([10.0, 20.0, sp[2], sp[3], 50.0, 60.0])
    assert np.allclose(se, want, rtol=1e-14, atol=0)


def _block_of_pixel(y, x, hb, wb):
    """The block whose 8x8 pixel rectangle holds (y, x), by search."""
    for by in range(hb):
        if 8 * by <= y < 8 * by + 8:
            for bx in range(wb):
                if 8 * bx <= x < 8 * bx + 8:
                    return by, bx
    raise AssertionError("no block")


@pytest.mark.parametrize("h,w,s,c,K", [(200, 300, 4, 3, 16), (137, 263, 3, 1, 32), (64, 64, 5, 3, 8)])
def test_effective_map_and_tau_by_brute_force(h, w, s, c, K):
    rng = np.random.default_rng(h + w)
    hb, wb = -(-h // 8), -(-w // 8)
    nty, ntx = est.tile_grid(h, w)
    z = rng.normal(np.log(30.0), 0.3, (hb, wb))
    use_plain = rng.random(nty * ntx) < 0.4
    sig_hat = rng.uniform(10, 50, nty * ntx)
    factor = np.where(rng.random(nty * ntx) < 0.5, 1.0 / 1.2, 1.0)
    smap = est.effective_sigma_map(h, w, sig_hat, z=z, use_plain=use_plain, factor=factor)
    mult = oracle.tau_multiplier(c, K)
    tau = est.tau_from_sigma_map(smap, h, w, 8, s, c, K)
    ys, xs = oracle.ref_grid(h, 8, s), oracle.ref_grid(w, 8, s)
    r = 0
    for y in ys:
        for x in xs:
            t = (int(y) // 128) * ntx + int(x) // 128          # tile of the top-left pixel
            by, bx = _block_of_pixel(int(y), int(x), hb, wb)
            want = sig_hat[t] if use_plain[t] else math.exp(z[by, bx]) * factor[t]
            assert math.isclose(tau[r], want * mult, rel_tol=1e-15), (y, x)
            r += 1
    assert r == tau.size


def test_vote_factor_majority():
    votes = np.array([8, 7, 3, 2, 0, 15])
    nvotes = np.array([15, 15, 5, 4, 0, 15])
    assert list(est.vote_factor(votes, nvotes, 1.2)) == [1 / 1.2, 1.0, 1 / 1.2, 1.0, 1.0, 1 / 1.2]


def test_all_tiles_rejecting_reduces_to_the_plain_rule():
    """A map far from every plain estimate is rejected everywhere: the thresholds are those of
    the plain estimate with the Eq. 23 vote (the existing plain-path oracle)."""
    clean, noisy, _ = synth.make_cfg("rgb512_awgn50", h=140, w=200)
    h, w = noisy.shape[:2]
    ps, s, W, K = 8, 4, 15, 16
    z = np.full((-(-h // 8), -(-w // 8)), 12.0)          # sigma = e^12
    got = est.thresholds(noisy, ps, s, W, K, z=z)
    assert got["use_plain"].all()
    idx, _ = oracle.block_match(noisy, ps, s, W, K)
    se = est.sigma_est_tiles(noisy)
    sh = est.sigma_hat_tiles(noisy, idx, se, ps, s)
    want = est.tau_per_ref(sh, h, w, ps, s, 3, K)
    assert np.allclose(got["tau"], want, rtol=1e-15, atol=0)
    plain = est.thresholds(noisy, ps, s, W, K)
    assert np.array_equal(plain["tau"], got["tau"])


def test_constant_map_accepted_gives_its_level():
    """Flat image with AWGN sigma 20 (the plain estimate is within 3% of 20): a map constant at
    sigma 21 is kept on every tile, so each reference's tau is 21 times its tile's vote factor."""
    rng = np.random.default_rng(5)
    h, w = 192, 256
    img = np.clip(np.rint(120.0 + rng.normal(0, 20.0, (h, w, 3))), 0, 255).astype(np.uint8)
    z = np.full((h // 8, w // 8), math.log(21.0))
    got = est.thresholds(img, 8, 4, 15, 16, z=z)
    assert not got["use_plain"].any()
    assert np.allclose(got["sigma_est"], 21.0, rtol=1e-14)
    f = est.vote_factor(got["votes"], got["nvotes"])
    tile_of = est.tile_of_refs(oracle.ref_grid(h, 8, 4), oracle.ref_grid(w, 8, 4), h, w)
    assert np.allclose(got["tau"], 21.0 * f[tile_of] * oracle.tau_multiplier(3, 16), rtol=1e-14)


def test_restricted_tiles_agree_with_the_whole_image():
    clean, noisy, _ = synth.make_cfg("rgb512_awgn50", h=260, w=300)
    h, w = noisy.shape[:2]
    rng = np.random.default_rng(3)
    z = rng.normal(np.log(50.0), 0.2, (-(-h // 8), -(-w // 8)))
    full = est.thresholds(noisy, 8, 4, 15, 16, z=z)
    part = est.thresholds(noisy, 8, 4, 15, 16, z=z, tiles=[1, 5])
    for key in ("sigma_est", "sigma_hat", "votes"):
        assert np.array_equal(part[key][[1, 5]], full[key][[1, 5]])
    ok = ~np.isnan(part["tau"])
    assert ok.any() and np.array_equal(part["tau"][ok], full["tau"][ok])
    assert np.isnan(part["sigma_est"][0])


def test_auto_group_size_cutoff_is_strict():
    assert est.auto_group_size([30.0, 30.0], 30.0) == 32
    assert est.auto_group_size([20.0, math.nextafter(40.0, 0.0)], 30.0) == 16
    assert est.auto_group_size([10.0, 50.0], 30.5) == 16
    assert est.auto_group_size([10.0, 52.0], 30.5) == 32
