"""The warm-start network's GPU kernels (BF16 matrix cores, FP32 accumulation)
against the FP64 CPU reference of oracle/mlp_ref.py.

Bars: with the reference rounding to BF16 at the same points as the kernels,
forward outputs agree to 2e-3 relative (only the accumulation order differs)
and parameter gradients to 2e-2 relative L2 per layer; against the plain FP64
reference (no BF16 rounding) to 3e-2 / 1e-1.
"""
import numpy as np
import pytest

from oracle import mlp_ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _setup(torch, n_in=128, width=64, n_out=64, rows=100, seed=3):
    from paper_2001_10986_amd import mlp
    net = mlp.MLP(n_in, n_out, width, seed=seed)
    rng = np.random.default_rng(seed)
    p = net.get_params().astype(np.float64)
    p += rng.normal(size=p.size) * 0.01  # non-zero biases
    net.set_params(p.astype(np.float32))
    p = net.get_params().astype(np.float64)
    x = rng.normal(size=(rows, n_in)).astype(np.float32)
    t = rng.normal(size=(rows, n_out)).astype(np.float32)
    m = (rng.uniform(size=(rows, n_out)) > 0.2).astype(np.float32)
    d = lambda a: torch.from_numpy(a).cuda()
    return net, p, x, t, m, d


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def test_forward_matches_reference(torch):
    net, p, x, t, m, d = _setup(torch)
    y = net.forward(d(x)).cpu().numpy().astype(np.float64)
    yq = mlp_ref.forward(p, net.dims, x, bf16=True)[0]
    y64 = mlp_ref.forward(p, net.dims, x, bf16=False)[0]
    assert _rel(y, yq) < 2e-3
    assert _rel(y, y64) < 3e-2


def test_gradients_match_reference(torch):
    net, p, x, t, m, d = _setup(torch)
    loss, g = net.loss_grad(d(x), d(t), d(m))
    lq, gq = mlp_ref.loss_grad(p, net.dims, x, t, m, bf16=True)
    l64, g64 = mlp_ref.loss_grad(p, net.dims, x, t, m, bf16=False)
    assert abs(loss - lq) < 2e-3 * lq and abs(loss - l64) < 3e-2 * l64
    off = 0
    for l in range(4):
        n = net.dims[l] * net.dims[l + 1] + net.dims[l + 1]
        sl = slice(off, off + n)
        off += n
        assert _rel(g[sl], gq[sl]) < 2e-2, l
        assert _rel(g[sl], g64[sl]) < 1e-1, l


def test_training_reduces_the_loss(torch):
    from paper_2001_10986_amd import mlp
    rng = np.random.default_rng(4)
    net = mlp.MLP(64, 64, 64, seed=5)
    A = rng.normal(size=(64, 64)) / 8
    x = rng.normal(size=(512, 64)).astype(np.float32)
    t = np.tanh(x @ A).astype(np.float32)
    m = np.ones_like(t)
    xd, td, md = (torch.from_numpy(a).cuda() for a in (x, t, m))
    first = net.train_step(xd, td, md, 3e-3)
    for _ in range(300):
        last = net.train_step(xd, td, md, 3e-3)
    assert last < 0.1 * first
