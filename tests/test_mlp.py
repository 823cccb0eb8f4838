"""The CPU reference of the picker network, pinned: its analytic gradient
against central finite differences, its Adam step against the closed form of
the first step."""
import numpy as np
import pytest

from oracle import mlp


def _data(seed, nb=16):
    r = np.random.default_rng([50, seed])
    p = r.normal(0, 0.3, mlp.count())
    X = r.normal(0, 1, (nb, 4))
    T = r.normal(0, 1, (nb, 45))
    mask = (r.uniform(size=(nb, 45)) < 0.8).astype(float)
    return p, X, T, mask


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_finite_differences(seed):
    p, X, T, mask = _data(seed)
    g = mlp.grad(p, X, T, mask)
    r = np.random.default_rng([51, seed])
    idx = r.choice(mlp.count(), 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, X, T, mask) - mlp.loss(p - e, X, T, mask)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, (i, fd, g[i])


def test_layout_and_count():
    assert mlp.count() == 4 * 64 + 64 + 64 * 64 + 64 + 45 * 64 + 45
    p = np.arange(mlp.count(), dtype=float)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    assert W1.shape == (64, 4) and W1[0, 1] == 1 and b1[0] == 256
    assert W3.shape == (45, 64) and b3[-1] == mlp.count() - 1


def test_adam_first_step_closed_form():
    r = np.random.default_rng(52)
    p = r.normal(size=100)
    g = r.normal(size=100)
    lr = 0.01
    p1, m, v = mlp.adam(p, g, np.zeros(100), np.zeros(100), 1, lr=lr, eps=0.0)
    assert np.allclose(p1, p - lr * np.sign(g), rtol=0, atol=1e-15)


def test_zero_mask_gives_zero_gradient():
    p, X, T, mask = _data(3)
    assert np.all(mlp.grad(p, X, T, np.zeros_like(mask)) == 0)
