"""The warm-start network's GPU kernels (BF16 matrix cores, FP32 accumulation)
against the FP64 CPU reference of oracle/mlp_ref.py.

Element-wise bars.  The reference rounds to BF16 at the same points as the
kernels and accumulates in FP64; the kernels accumulate in FP32, so an
intermediate BF16 value can round to the neighbouring BF16 number (one unit
of 2^-8 relative).  Along any path from the inputs to an output there are at
most 3 such rounding points in the forward pass and 8 in the backward pass,
so, to first order, an output differs from the reference by at most
3 * 2^-8 times its magnitude |x| |W1| + |b1| ... |W4| + |b4| (the sum
without cancellation), and a weight gradient by at most 8 * 2^-8 = 2^-5
times |h_l|^T |g_l| (the same without cancellation).  Without any such
rounding flip the only difference is the FP32 accumulation of at most 256
products per sum, K * 2^-24 < 2e-5 relative; the relative L2 bars are set
there (measured 4e-8 on these inputs, which round identically on both
sides) and the plain FP64 reference (no BF16 rounding) is bounded by the
BF16 rounding itself.
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


def _magnitude(p, dims, x):
    """|x| |W1| + |b1|, ... through the four layers (an upper bound of every
    pre-activation's size; ReLU only shrinks)."""
    m = np.abs(mlp_ref.bf16_round(x))
    for W, b in mlp_ref.unflatten(p, dims):
        m = m @ np.abs(mlp_ref.bf16_round(W)) + np.abs(b)
    return m


def test_forward_matches_reference(torch):
    net, p, x, t, m, d = _setup(torch)
    y = net.forward(d(x)).cpu().numpy().astype(np.float64)
    yq = mlp_ref.forward(p, net.dims, x, bf16=True)[0]
    y64 = mlp_ref.forward(p, net.dims, x, bf16=False)[0]
    mag = _magnitude(p, net.dims, x)
    err = np.abs(y - yq)
    print("forward: max |y - ref| / bound", (err / (3 * 2.0 ** -8 * mag)).max(),
          "rel L2", _rel(y, yq), flush=True)
    assert np.all(err <= 3 * 2.0 ** -8 * mag + 1e-6)
    assert _rel(y, yq) < 2e-5
    assert _rel(y, y64) < 3e-2


def test_gradients_match_reference(torch):
    net, p, x, t, m, d = _setup(torch)
    loss, g = net.loss_grad(d(x), d(t), d(m))
    lq, gq = mlp_ref.loss_grad(p, net.dims, x, t, m, bf16=True)
    l64, g64 = mlp_ref.loss_grad(p, net.dims, x, t, m, bf16=False)
    assert abs(loss - lq) < 2e-5 * lq and abs(loss - l64) < 3e-2 * l64
    # magnitudes without cancellation: |h_l|^T |g_l| for the weights and
    # sum |g_l| for the biases, g_l the back-propagated output gradient
    _, acts, zs = mlp_ref.forward(p, net.dims, x, bf16=True)
    layers = mlp_ref.unflatten(p, net.dims)
    gm = np.abs(2.0 * m * (mlp_ref.forward(p, net.dims, x, bf16=True)[0] - t) / m.sum())
    bounds = [None] * 4
    for l in range(3, -1, -1):
        bounds[l] = np.concatenate([(np.abs(acts[l]).T @ gm).ravel(), gm.sum(axis=0)])
        if l > 0:
            gm = (gm @ np.abs(mlp_ref.bf16_round(layers[l][0])).T) * (zs[l - 1] > 0)
    off = 0
    for l in range(4):
        n = net.dims[l] * net.dims[l + 1] + net.dims[l + 1]
        sl = slice(off, off + n)
        off += n
        err = np.abs(g[sl] - gq[sl])
        print(f"layer {l}: max |g - ref| / bound {(err / (2.0 ** -5 * bounds[l] + 1e-12)).max():.3g}, "
              f"rel L2 {_rel(g[sl], gq[sl]):.3g}", flush=True)
        assert np.all(err <= 2.0 ** -5 * bounds[l] + 1e-9), l
        assert _rel(g[sl], gq[sl]) < 2e-5, l
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
