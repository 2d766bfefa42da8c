"""Pins of the FP64 oracle of the sigma-map network (no GPU)."""
import numpy as np
import pytest
import scipy.signal

from oracle import cnn


def _rand_params(c, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(cnn.n_params(c)) * scale


@pytest.mark.parametrize("s", [1, 2])
def test_conv_matches_scipy_correlate(s):
    rng = np.random.default_rng(s)
    x = rng.standard_normal((2, 11, 14, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = cnn.conv_forward(x, w, b, s)
    for n in range(2):
        for co in range(4):
            acc = np.full((11, 14), b[co])
            for ci in range(3):
                xp = np.pad(x[n, :, :, ci], 1)
                acc = acc + scipy.signal.correlate2d(xp, w[co, :, :, ci], mode="valid")
            assert np.allclose(y[n, :, :, co], acc[::s, ::s], atol=1e-12)
    assert y.shape[1:3] == (-(-11 // s), -(-14 // s))


def test_output_is_one_value_per_8x8_block():
    x = np.random.default_rng(0).integers(0, 256, (1, 40, 27, 3))
    z, _ = cnn.forward(_rand_params(3, 1), x, 3)
    assert z.shape == (1, 5, 4)


@pytest.mark.parametrize("c", [1, 3])
def test_gradient_matches_central_differences(c):
    rng = np.random.default_rng(c)
    x = rng.integers(0, 256, (2, 24, 16, c))
    flat = _rand_params(c, 10 + c)
    tgt = rng.uniform(1.0, 4.0, (2, 3, 2))
    loss, g = cnn.loss_and_grad(flat, x, tgt, c)
    idx = rng.choice(flat.size, 60, replace=False)
    eps = 1e-6
    num = []
    for i in idx:
        f = flat.copy()
        f[i] += eps
        lp, _ = cnn.loss_and_grad(f, x, tgt, c)
        f[i] -= 2 * eps
        lm, _ = cnn.loss_and_grad(f, x, tgt, c)
        num.append((lp - lm) / (2 * eps))
    num = np.array(num)
    ana = g[idx]
    err = np.abs(num - ana)
    assert np.all(err <= 1e-6 + 1e-5 * np.abs(ana)), (err.max(), num, ana)


def test_block_targets_constant_and_rms():
    f = np.full((20, 13), 7.0)
    assert np.allclose(cnn.block_targets(f), np.log(7.0))
    f = np.zeros((8, 8))
    f[:4] = 3.0
    f[4:] = 4.0
    assert np.isclose(cnn.block_targets(f)[0, 0], 0.5 * np.log((9 + 16) / 2))


def test_flatten_roundtrip():
    flat = _rand_params(3, 5)
    assert np.array_equal(cnn.flatten(cnn.unflatten(flat, 3)), flat)
    assert cnn.n_params(3) == 32 * 27 + 32 + 4 * (32 * 288 + 32) + 288 + 1
