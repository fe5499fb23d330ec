"""dd_cost_noalloc (the allocation-free diagnostics) against dd_cost through
the C-ABI: two calls in a row, the second on a smaller level (the shared
static scratch keeps the first call's contents, so the second must clear
what it uses), and the size limit of the static scratch."""
import numpy as np
import pytest

from paper_2001_10986_amd import datagen

pytestmark = pytest.mark.gpu

EXACT = ("cost", "obj", "err_x", "nnz", "level", "last_partition", "eps")


def _same_report(a, b):
    for k in EXACT:
        assert a[k] == b[k], (k, a[k], b[k])
    # err_y and the drift sum per-pixel marginals accumulated with atomics:
    # the same values up to the order of the additions
    assert abs(a["err_y"] - b["err_y"]) <= 1e-15 + 1e-12 * b["err_y"]
    assert abs(a["mass_drift"] - b["mass_drift"]) <= 1e-15 + 1e-12 * b["mass_drift"]


def test_noalloc_cost_matches_cost_on_two_calls():
    from paper_2001_10986_amd import dd
    big = datagen.small_pair(64, 4, seed=17)
    small = datagen.small_pair(32, 3, seed=5)
    probs = []
    for (mu, nu), N in ((big, 64), (small, 32)):
        g = dd.Problem(mu, nu, [(0, 4.0 / N ** 2, 3)], s=4, n_levels=1)
        for ell in range(3):
            g.half_iterate(ell % 2)
        probs.append(g)
    # first call on the 64x64 level fills 4096 accumulator slots, the second
    # (32x32, 1024 slots) must not see them
    r_big = probs[0].cost_noalloc()
    r_small = probs[1].cost_noalloc()
    _same_report(r_big, probs[0].cost())
    _same_report(r_small, probs[1].cost())
    assert r_small["err_y"] < 1e-5 and r_big["err_y"] < 1e-5
    # and again in the other order, after the allocating calls
    _same_report(probs[1].cost_noalloc(), probs[1].cost())
    _same_report(probs[0].cost_noalloc(), probs[0].cost())
    for g in probs:
        g.close()


def test_noalloc_cost_rejects_levels_above_its_scratch():
    # a 2304 x 2048 finest level (4 718 592 pixels > 2^22): the state is
    # imported directly at that level (every basic cell keeps its own pixels)
    from paper_2001_10986_amd import dd
    H, W, s, nlev = 2304, 2048, 4, 6
    mu = np.full((H, W), 1.0 / (H * W))
    g = dd.Problem(mu, mu, [(nlev - 1, 1e-6, 2)], s=s, n_levels=nlev)
    bh, bw = H // s, W // s
    nb = bh * bw
    br, bc = np.divmod(np.arange(nb), bw)
    ii, jj = np.divmod(np.arange(s * s), s)
    col = ((br[:, None] * s + ii[None, :]) * W + bc[:, None] * s + jj[None, :]).astype(np.int32)
    view = {"level": nlev - 1, "eps": 1e-6, "row_ptr": np.arange(nb + 1, dtype=np.int64) * s * s,
            "col": col.ravel(), "val": mu.ravel()[col.ravel()],
            "alpha_a": np.zeros((H, W)), "alpha_b": np.zeros((H, W))}
    g.import_state(**view)
    with pytest.raises(dd.DDError, match="static"):
        g.cost_noalloc()
    r = g.cost()
    assert r["level"] == nlev - 1 and r["nnz"] == H * W and r["err_y"] < 1e-12
    g.close()
