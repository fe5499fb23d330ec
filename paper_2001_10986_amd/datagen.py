"""Seeded synthetic inputs: Gaussian-blob image pairs and eps schedules.

This module holds none of the method's arithmetic.  It draws the test images
(the paper's are random Gaussian mixtures, Sec. 7.1 "Test data"; they are not
published, so these stand in for them) and writes out the stage lists that the
driver runs.  Both the GPU path and the oracle take their inputs from here.

Recipe for one image of H x W pixels with n blobs (seed s):
  rng = numpy.random.default_rng(s); for each blob draw, in this order,
  centre x ~ U[0,1], centre y ~ U[0,1], std ~ U[0.03,0.15], amplitude ~ U[0.5,1];
  density(p) = sum_blobs a * exp(-|p - c|^2 / (2 std^2)) at the pixel centres
  p = ((col+1/2) h, (row+1/2) h), h = 1/max(H,W); then either add a floor of
  floor*max (default 1e-3) or i.i.d. noise U[0, noise]*max per pixel; finally
  normalise to total mass 1.
"""
import numpy as np


def blob_image(H, W, n_blobs, seed, floor=1e-3, noise=0.0):
    rng = np.random.default_rng(seed)
    h = 1.0 / max(H, W)
    yy = (np.arange(H) + 0.5) * h
    xx = (np.arange(W) + 0.5) * h
    img = np.zeros((H, W))
    for _ in range(n_blobs):
        cx, cy, sd, a = rng.uniform(0, 1), rng.uniform(0, 1), rng.uniform(0.03, 0.15), \
            rng.uniform(0.5, 1.0)
        img += a * np.exp(-((xx[None, :] - cx) ** 2 + (yy[:, None] - cy) ** 2) / (2 * sd * sd))
    mx = img.max()
    if noise > 0:
        img += rng.uniform(0.0, noise, size=(H, W)) * mx
    else:
        img += floor * mx
    return img / img.sum()


def eps_schedule(N, n_levels, eps_start=1.0, final_eps=None, p=2.0, level_factor=0.5):
    """Stage list [(level, eps, n_half_iterations)] of the multi-scale eps-scaling driver.

    Follows Sec. 7.1 ("Multi-scale and eps-scaling") in unit coordinates: on
    level l (pixel spacing h_l) eps halves from stage to stage while
    eps >= h_l^2/2; the first stage of a level runs 4 half-iterations
    (A,B,A,B), later ones 2; the next level starts at the last eps of the
    previous one (h_l^2/2 = 2 h_{l+1}^2).  On the finest level eps stops at
    final_eps (default h^2) and 2 more half-iterations run there.  For a cost
    |x-y|^p the thresholds are level_factor * h_l^p (default h_l^p / 2) and
    the default final eps h^p.
    """
    if final_eps is None:
        final_eps = (1.0 / N) ** p
    stages = []
    eps = float(eps_start)
    for lev in range(n_levels):
        Nl = N >> (n_levels - 1 - lev)
        lo = level_factor / Nl ** p if lev < n_levels - 1 else final_eps
        first = True
        while eps >= lo * (1 - 1e-12):
            stages.append([lev, eps, 4 if first else 2])
            first = False
            eps *= 0.5
        eps *= 2.0
        if first:  # eps already below this level's range: run one stage at it
            stages.append([lev, eps, 4])
    stages[-1][2] += 2
    return [tuple(s) for s in stages]


def paper_schedule(N, coarsest=8, final_factor=0.25):
    """Stage list of the paper's own protocol (Sec. 7.1 "Multi-scale and
    eps-scaling"), in unit coordinates: layers from a coarsest side of
    `coarsest` pixels up to N; on each layer with pixel spacing h_l, 4
    half-iterations at eps = 2 h_l^2, then 2 at h_l^2 and 2 at h_l^2/2, then
    refinement; on the finest layer 2 more at final_factor * h^2 (the paper:
    a quarter of the squared pixel spacing).  Returns (stages, n_levels)."""
    n_levels = int(round(np.log2(N // coarsest))) + 1
    if coarsest << (n_levels - 1) != N:
        raise ValueError("N must be coarsest * 2^k")
    stages = []
    for lev in range(n_levels):
        h2 = (1.0 / (coarsest << lev)) ** 2
        stages += [(lev, 2.0 * h2, 4), (lev, h2, 2), (lev, 0.5 * h2, 2)]
    stages.append((n_levels - 1, final_factor / N ** 2, 2))
    return stages, n_levels


# --- the benchmark configurations (image k of config c uses seed 1000*c + k) ---

def config1_pair():
    """32x32 pair, 4 blobs, floor 1e-3*max; single level, eps = 4/32^2, 40 half-iterations."""
    mu = blob_image(32, 32, 4, 1000)
    nu = blob_image(32, 32, 4, 1001)
    return mu, nu, dict(s=4, n_levels=1, stages=[(0, 4.0 / 32 ** 2, 40)])


def config2_pair(i=0, j=1):
    """256x256 pair (images i, j of 10), 8 blobs; levels 64->128->256, eps 1 -> (1/256)^2."""
    mu = blob_image(256, 256, 8, 2000 + i)
    nu = blob_image(256, 256, 8, 2000 + j)
    return mu, nu, dict(s=4, n_levels=3, stages=eps_schedule(256, 3))


def config3_pair(seed0=3000, N=1024, final_factor=1.0):
    """NxN pair (default 1024), 16 blobs + U[0,0.1]*max noise; levels 64->N,
    eps 1 -> final_factor*(1/N)^2.  N = 2048 with final_factor = 0.25 is the
    paper's largest image size (summary table of the quantitative evaluation)
    and its final eps of a quarter pixel spacing squared (Sec. 7.1)."""
    if N < 64 or N & (N - 1):
        raise ValueError("N must be a power of two >= 64")
    nlev = int(np.log2(N // 64)) + 1
    mu = blob_image(N, N, 16, seed0, noise=0.1)
    nu = blob_image(N, N, 16, seed0 + 1, noise=0.1)
    return mu, nu, dict(s=4, n_levels=nlev,
                        stages=eps_schedule(N, nlev, final_eps=final_factor / N ** 2))


def config4_pairs(n_pairs=64, sizes=(64, 128, 256, 512)):
    """Uneven batch: n_pairs independent pairs, side drawn uniformly from `sizes`,
    4-16 blobs per image (floor 1e-3*max); sides and blob counts come from
    default_rng(4000), image k (2 per pair) from seed 4001 + k.  Each pair runs
    its own multi-scale schedule from a 64x64 coarsest level to (1/N)^2.
    Returns a list of (mu, nu, cfg)."""
    rng = np.random.default_rng(4000)
    out = []
    for k in range(n_pairs):
        N = int(rng.choice(sizes))
        nb = int(rng.integers(4, 17))
        nlev = int(np.log2(N // 64)) + 1 if N >= 64 else 1
        mu = blob_image(N, N, nb, 4001 + 2 * k)
        nu = blob_image(N, N, nb, 4002 + 2 * k)
        out.append((mu, nu, dict(s=4, n_levels=nlev, stages=eps_schedule(N, nlev))))
    return out


def small_pair(N, n_blobs=4, seed=7, n_levels=1):
    mu = blob_image(N, N, n_blobs, seed)
    nu = blob_image(N, N, n_blobs, seed + 1)
    return mu, nu
