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


def test_adam_first_step_closed_form():
    """Step 1: the corrected moments are g and g^2, so every parameter moves by
    lr * g / (|g| + eps) (Kingma and Ba 2015, Algorithm 1)."""
    rng = np.random.default_rng(0)
    w0 = rng.standard_normal(50)
    g = rng.standard_normal(50) * 10.0 ** rng.uniform(-9, 1, 50)
    w1, m1, v1 = cnn.adam_step(w0, np.zeros(50), np.zeros(50), g, 1, 1e-3)
    assert np.allclose(w1, w0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-13, atol=1e-18)
    assert np.allclose(m1, 0.1 * g, rtol=1e-15) and np.allclose(v1, 0.001 * g * g, rtol=1e-13)


def test_adam_constant_gradient_moves_by_lr_per_step():
    """With the same gradient every step the bias correction makes the corrected moments
    exactly g and g^2, so each step moves by the same lr * g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 3e-3, -1e-6])
    w = np.zeros(4)
    m = v = np.zeros(4)
    for t in range(1, 30):
        w_prev = w
        w, m, v = cnn.adam_step(w, m, v, g, t, 0.01)
        assert np.allclose(w - w_prev, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=0)


def test_adam_matches_torch_adam_in_fp64():
    """Against PyTorch's own Adam (an independent implementation), FP64 on the CPU."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    w0 = rng.standard_normal(64)
    p = torch.nn.Parameter(torch.tensor(w0, dtype=torch.float64))
    opt = torch.optim.Adam([p], lr=2e-3, betas=(0.9, 0.999), eps=1e-8)
    w, m, v = w0, np.zeros(64), np.zeros(64)
    for t in range(1, 8):
        g = rng.standard_normal(64) * (0.1 * t)
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        w, m, v = cnn.adam_step(w, m, v, g, t, 2e-3)
        assert np.allclose(p.detach().numpy(), w, rtol=1e-13, atol=1e-15)
