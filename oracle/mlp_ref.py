"""Plain NumPy FP64 reference of the warm-start network (forward, masked MSE
loss, gradients).

TEST INFRASTRUCTURE ONLY: the tests use it to check the GPU network's forward
pass and gradients; the product path never imports it.

Network: y = L4(relu(L3(relu(L2(relu(L1(x))))))), L_l(h) = h W_l + b_l,
parameters flat in the order W_1, b_1, ..., W_4, b_4 (W row-major, in x out).
Loss: L = sum mask (y - t)^2 / sum mask.  With `bf16=True` the reference
rounds to BF16 (nearest even) at the points where the GPU kernels store BF16:
the inputs, the weights, the hidden activations after ReLU, and the
back-propagated gradients that enter a matrix product.
"""
import numpy as np


def bf16_round(a):
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unflatten(params, dims):
    out, off = [], 0
    for l in range(4):
        W = params[off:off + dims[l] * dims[l + 1]].reshape(dims[l], dims[l + 1])
        off += dims[l] * dims[l + 1]
        b = params[off:off + dims[l + 1]]
        off += dims[l + 1]
        out.append((np.asarray(W, np.float64), np.asarray(b, np.float64)))
    return out


def forward(params, dims, x, bf16=False):
    q = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    layers = unflatten(params, dims)
    h = q(x)
    acts, zs = [h], []
    for l, (W, b) in enumerate(layers):
        z = h @ q(W) + b
        zs.append(z)
        if l < 3:
            h = q(np.maximum(z, 0.0))
            acts.append(h)
    return z, acts, zs


def loss_grad(params, dims, x, t, mask, bf16=False):
    q = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    y, acts, zs = forward(params, dims, x, bf16)
    cnt = mask.sum()
    diff = y - t
    loss = float((mask * diff * diff).sum() / cnt)
    g = q(2.0 * mask * diff / cnt)
    layers = unflatten(params, dims)
    grads = [None] * 4
    for l in range(3, -1, -1):
        W, _ = layers[l]
        grads[l] = (acts[l].T @ g, g.sum(axis=0))
        if l > 0:
            dh = g @ q(W).T
            g = q(dh * (zs[l - 1] > 0))
    flat = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])
    return loss, flat
