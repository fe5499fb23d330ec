"""Pins of the CPU reference of the warm-start network (CPU only)."""
import numpy as np

from oracle import mlp_ref


def _net(seed=0):
    rng = np.random.default_rng(seed)
    dims = [8, 6, 6, 6, 4]
    n = sum(dims[l] * dims[l + 1] + dims[l + 1] for l in range(4))
    return dims, rng.normal(size=n) * 0.7, rng


def test_gradient_matches_central_differences():
    dims, p, rng = _net(1)
    x = rng.normal(size=(5, 8))
    t = rng.normal(size=(5, 4))
    mask = (rng.uniform(size=(5, 4)) > 0.3).astype(float)
    loss, g = mlp_ref.loss_grad(p, dims, x, t, mask)
    h = 1e-6
    num = np.empty_like(p)
    for k in range(len(p)):
        e = np.zeros_like(p)
        e[k] = h
        num[k] = (mlp_ref.loss_grad(p + e, dims, x, t, mask)[0] -
                  mlp_ref.loss_grad(p - e, dims, x, t, mask)[0]) / (2 * h)
    assert np.abs(num - g).max() < 1e-7 * max(1.0, np.abs(g).max())


def test_forward_is_the_composition_written_out():
    dims, p, rng = _net(2)
    x = rng.normal(size=(3, 8))
    L = mlp_ref.unflatten(p, dims)
    h = x
    for l, (W, b) in enumerate(L):
        h = h @ W + b
        if l < 3:
            h = np.where(h > 0, h, 0.0)
    assert np.allclose(mlp_ref.forward(p, dims, x)[0], h, rtol=1e-13, atol=1e-13)


def test_bf16_rounding_is_nearest_even():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0], dtype=np.float32)
    r = mlp_ref.bf16_round(v)
    assert r[0] == 1.0 and r[1] == 1.0  # tie -> even
    assert r[2] == 1.0 + 2 ** -7 and r[3] == -2.5 and r[4] == 0.0
