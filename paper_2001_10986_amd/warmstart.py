"""Learned warm start: data from the plain method, GPU training, evaluation.

The network (paper_2001_10986_amd.mlp.MLP, 768 -> 256 -> 256 -> 256 -> 64)
maps the features of a composite cell problem (mu_J, nu_J, eps and the
potential the solve would start from; see include/dd_mlp.h) to the change
that the cell solve makes to that potential.  Training samples are the cell
problems that the plain GPU method solves on 256x256 image pairs of the blob
generator (8 blobs, 3 levels, the same eps schedule as the other workloads).  Everything runs in the
library's kernels; this module only drives them.
"""
import numpy as np
import torch

from . import datagen, dd, mlp

N_IN, N_OUT, WIDTH = 768, 64, 256
# default use: on the first sweep of each partition after dd_init or dd_refine
# (policy 3), for cells whose predicted change has RMS >= MIN_RMS (units of
# 16 h^2/eps); on the 1024x1024 workload the best of policies 1-3 with
# thresholds {0, 0.25, 0.5, 1}, by a small margin (all within ~3 %)
POLICY, MIN_RMS = 3, 0.5


def training_pair(k):
    """Image pair k of the training set (seed block 2000 + k, distinct from the
    evaluation pairs)."""
    mu = datagen.blob_image(256, 256, 8, 2000 + 2 * k)
    nu = datagen.blob_image(256, 256, 8, 2000 + 2 * k + 1)
    return mu, nu, datagen.eps_schedule(256, 3)


def generate(n_pairs, cap, device="cuda", log=None):
    """Run the plain method on n_pairs training pairs and collect every
    converged eligible cell problem (at most cap samples)."""
    X = torch.empty((cap, N_IN), dtype=torch.float32, device=device)
    T = torch.empty((cap, N_OUT), dtype=torch.float32, device=device)
    M = torch.empty((cap, N_OUT), dtype=torch.float32, device=device)
    n = 0
    for k in range(n_pairs):
        mu, nu, sched = training_pair(k)
        g = dd.Problem(torch.from_numpy(mu).to(device), torch.from_numpy(nu).to(device), sched,
                       s=4, n_levels=3)
        for (lev, eps, nh) in sched:
            while g.level_info()["level"] < lev:
                g.refine()
            g.set_eps(eps)
            for h in range(nh):
                g.half_iterate(h & 1)
                if n < cap:
                    n += g.collect_cells(X[n:], T[n:], M[n:])
        g.close()
        if log:
            log(f"pair {k}: {n} samples")
        if n >= cap:
            break
    return X[:n], T[:n], M[:n]


def train(net, X, T, M, steps, batch=4096, lr=1e-3, seed=0, log=None):
    """Adam on random minibatches with a cosine-decayed learning rate."""
    gen = torch.Generator(device=X.device)
    gen.manual_seed(seed)
    n = X.shape[0]
    losses = []
    for s in range(steps):
        idx = torch.randint(0, n, (batch,), device=X.device, generator=gen)
        rate = lr * 0.5 * (1 + np.cos(np.pi * s / steps))
        losses.append(net.train_step(X[idx].contiguous(), T[idx].contiguous(),
                                     M[idx].contiguous(), max(rate, lr * 1e-3)))
        if log and (s % 200 == 0 or s == steps - 1):
            log(f"step {s}: loss {losses[-1]:.4g}")
    return losses


def mean_loss(net, X, T, M, batch=8192):
    """Masked MSE of the network on a sample set (no update)."""
    tot, cnt = 0.0, 0.0
    for a in range(0, X.shape[0], batch):
        y = net.forward(X[a:a + batch].contiguous())
        d = (y - T[a:a + batch]) * M[a:a + batch]
        tot += float((d * d).sum())
        cnt += float(M[a:a + batch].sum())
    return tot / max(cnt, 1.0)
