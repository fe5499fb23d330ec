"""Pins of the sparse FP64 C oracle against the dense references and against
the exact invariants of the paper (CPU only)."""
import numpy as np
import pytest

from oracle import dense, ddo
from paper_2001_10986_amd import datagen


def _basic_marg_dense(plan, basic):
    return np.stack([plan[xs, :].sum(0) for xs in basic])


@pytest.mark.parametrize("cost_p", [1.5, 3.0])
def test_cell_solve_with_power_cost_matches_newton(cost_p):
    # c = |x-y|^p (strictly convex h, Sec. 7.1): the sparse cell solver
    # against the dense Newton solver of the same problem
    rng = np.random.default_rng(2)
    xr, xc = np.divmod(np.arange(64), 8)
    key = np.unique(rng.integers(0, 12, 35) * 12 + rng.integers(0, 12, 35))
    yr, yc = np.divmod(key, 12)
    mu = rng.uniform(0.5, 1, 64)
    nu = rng.uniform(0.5, 1, len(key))
    mu /= mu.sum()
    nu /= nu.sum()
    h = 1.0 / 16
    eps = 2.0 * h ** cost_p
    r = ddo.cell_solve(xr, xc, mu, yr, yc, nu, h ** cost_p / eps, 1e-13, 100000, cost_p=cost_p)
    d = np.sqrt((xr[:, None] - yr[None, :]) ** 2 + (xc[:, None] - yc[None, :]) ** 2)
    C = (d * h) ** cost_p
    P = dense.entropic_ot_newton(C, mu, nu, eps)[2]
    assert r["rc"] == 0
    assert np.abs(r["plan"] - P).max() < 1e-12


def test_cell_solve_matches_newton():
    # one composite cell of 8x8 pixels against a random 5x7 patch of Y points
    rng = np.random.default_rng(1)
    xr, xc = np.divmod(np.arange(64), 8)
    yr = rng.integers(0, 12, 35)
    yc = rng.integers(0, 12, 35)
    key = np.unique(yr * 12 + yc)
    yr, yc = np.divmod(key, 12)
    mu = rng.uniform(0.5, 1, 64)
    nu = rng.uniform(0.5, 1, len(key))
    mu /= mu.sum()
    nu /= nu.sum()
    h, eps = 1.0 / 16, 2.0 / 256
    r = ddo.cell_solve(xr, xc, mu, yr, yc, nu, h * h / eps, 1e-13, 100000)
    C = ((xr[:, None] - yr[None, :]) ** 2 + (xc[:, None] - yc[None, :]) ** 2) * h * h
    P = dense.entropic_ot_newton(C, mu, nu, eps)[2]
    assert r["rc"] == 0
    assert np.abs(r["plan"] - P).max() < 1e-12
    assert np.allclose(r["plan"].sum(0), nu, rtol=1e-13, atol=0)


@pytest.mark.parametrize("N,s,epsf,cost_p", [(8, 2, 2.0, 2.0), (16, 4, 4.0, 2.0),
                                              (16, 4, 4.0, 1.5), (16, 4, 4.0, 3.0)])
def test_half_iterations_match_dense_algorithm1(N, s, epsf, cost_p):
    mu, nu = datagen.small_pair(N, 3, seed=21)
    # (eps large enough that exp(-c/eps) stays above the FP64 range for
    # every pair of the grid, as the dense KL needs)
    eps = epsf / N ** cost_p * (4.0 if cost_p == 3.0 else 1.0)
    o = ddo.Oracle(mu, nu, s=s, n_levels=1, eps=eps, err_tol=1e-12, trunc=0.0, max_iter=100000,
                   cost_p=cost_p)
    basic, ca, cb = dense.grid_partitions(N, N, s)
    C = dense.grid_cost(N, N, 1.0 / N, p=cost_p)
    m, n = mu.ravel(), nu.ravel()
    pi0 = np.zeros((N * N, N * N))
    for xs in basic:
        pi0[xs, :] = np.outer(m[xs], n)
    n_half = 6
    plans = dense.dd_dense(C, m, n, eps, ca, cb, basic, pi0, n_half)
    K = dense.kernel(C, m, n, eps)
    prev_obj = np.inf
    for ell in range(n_half):
        st = o.half_iterate(ell % 2)
        bm = o.basic_marginals()
        assert np.abs(bm - _basic_marg_dense(plans[ell + 1], basic)).max() < 1e-11
        # reported transport cost and objective against the dense plan
        assert abs(st["cost"] - (C * plans[ell + 1]).sum()) < 1e-11
        obj_dense = eps * dense.kl(plans[ell + 1], K) - eps * K.sum()
        assert abs(st["obj"] - obj_dense) < 1e-10
        # the entropic objective never increases (proof of Proposition "SimpleConvergence")
        assert st["obj"] <= prev_obj + 1e-12
        prev_obj = st["obj"]


def test_converges_to_global_entropic_optimum():
    # the DD fixed point is the full-grid entropic optimum (Thm. "Linear convergence")
    N, s = 8, 2
    mu, nu = datagen.small_pair(N, 2, seed=31)
    eps = 32.0 / N ** 2
    o = ddo.Oracle(mu, nu, s=s, n_levels=1, eps=eps, err_tol=1e-12, trunc=0.0, max_iter=100000)
    C = dense.grid_cost(N, N, 1.0 / N)
    P = dense.entropic_ot_newton(C, mu.ravel(), nu.ravel(), eps)[2]
    basic, _, _ = dense.grid_partitions(N, N, s)
    target = _basic_marg_dense(P, basic)
    errs = []
    for ell in range(100):
        o.half_iterate(ell % 2)
        errs.append(np.abs(o.basic_marginals() - target).max())
    assert errs[-1] < 1e-9
    assert errs[-1] < errs[10] < errs[0]


def test_feasibility_invariants_with_truncation():
    mu, nu, cfg = datagen.config1_pair()
    o = ddo.Oracle(mu, nu, s=4, n_levels=1, eps=cfg["stages"][0][1], err_tol=1e-5, trunc=1e-15)
    for ell in range(6):
        st = o.half_iterate(ell % 2)
        r = o.cost()
        # |nu_i| = |mu_i| after BalanceMeasures, sum_i nu_i = nu (Algorithm 2 input
        # conditions) up to the truncated mass, X-error bounded by Err
        assert r["mass_drift"] <= 1e-13 + 1e-15 * r["nnz"]
        assert r["err_y"] <= 1e-13 + 1e-15 * r["nnz"] * 4
        assert st["err_x"] <= 1e-5 + 1e-15
        e = o.export()
        assert np.all(e["val"] >= 1e-15)
        for b in range(len(e["row_ptr"]) - 1):
            c = e["col"][e["row_ptr"][b]:e["row_ptr"][b + 1]]
            assert np.all(np.diff(c) > 0)


def test_balance_restores_masses_with_loose_tolerance():
    # a loose Sinkhorn tolerance leaves |nu_i| != |mu_i| after the split; the
    # balancing step must restore the masses without changing sum_i nu_i
    mu, nu = datagen.small_pair(16, 3, seed=41)
    o = ddo.Oracle(mu, nu, s=4, n_levels=1, eps=2.0 / 256, err_tol=1e-2, trunc=0.0)
    for ell in range(4):
        o.half_iterate(ell % 2)
        r = o.cost()
        assert r["mass_drift"] < 1e-15 * 64
        assert r["err_y"] < 1e-15 * 256
        assert np.all(o.export()["val"] > 0)


def test_refinement_invariants():
    # Proposition "FineBasicMarginals": sum_i nu_i^0 = nu and |nu_i^0| = mu(X_i)
    mu, nu = datagen.small_pair(32, 4, seed=51)
    o = ddo.Oracle(mu, nu, s=4, n_levels=2, eps=0.01, err_tol=1e-5, trunc=0.0)
    for ell in range(4):
        o.half_iterate(ell % 2)
    rc = o.cost()
    o.refine()
    info = o.level_info()
    assert (info["H"], info["level"]) == (32, 1)
    r = o.cost()
    # exact up to FP64 rounding (about 1e-16 per pixel) and what the coarse state carried
    assert r["err_y"] < 2 * rc["err_y"] + 1e-15 * 32 * 32
    assert r["mass_drift"] < 2 * rc["mass_drift"] + 1e-15 * 64
    e = o.export()
    assert e["val"].min() > 0


def test_refinement_glues_and_interpolates_potentials():
    # a globally consistent linear potential is reproduced exactly on the fine
    # grid, and arbitrary per-A-cell constants are removed by the gluing
    N, s = 32, 4
    mu, nu = datagen.small_pair(N, 4, seed=61)
    o = ddo.Oracle(mu, nu, s=s, n_levels=2, eps=0.01, err_tol=1e-5, trunc=1e-15)
    e = o.export()
    Hc = e["alpha_a"].shape[0]
    h = 1.0 / Hc
    rr, cc = np.meshgrid((np.arange(Hc) + 0.5) * h, (np.arange(Hc) + 0.5) * h, indexing="ij")
    f = 0.3 * rr - 0.7 * cc
    rng = np.random.default_rng(3)
    offs = rng.normal(size=(Hc // (2 * s), Hc // (2 * s))) * 0.05
    fa = f + np.kron(offs, np.ones((2 * s, 2 * s)))
    o.import_state(0, 0.01, e["row_ptr"], e["col"], e["val"], fa, f)
    o.refine()
    e2 = o.export()
    hf = 1.0 / (2 * Hc)
    rf, cf = np.meshgrid((np.arange(2 * Hc) + 0.5) * hf, (np.arange(2 * Hc) + 0.5) * hf,
                         indexing="ij")
    ff = 0.3 * rf - 0.7 * cf
    d = e2["alpha_a"] - ff
    assert np.abs(d - d.mean()).max() < 1e-12
    assert np.array_equal(e2["alpha_a"], e2["alpha_b"])


def test_eps_change_keeps_potentials():
    mu, nu, cfg = datagen.config1_pair()
    o = ddo.Oracle(mu, nu, s=4, n_levels=1, eps=0.01)
    o.half_iterate(0)
    a = o.export()["alpha_a"].copy()
    o.set_eps(0.005)
    assert np.array_equal(o.export()["alpha_a"], a)


def test_iteration_cap_is_reported():
    mu, nu, cfg = datagen.config1_pair()
    o = ddo.Oracle(mu, nu, s=4, n_levels=1, eps=cfg["stages"][0][1], max_iter=1, safeguard=1)
    st = o.half_iterate(0)
    assert st["n_failed"] > 0 and st["n_safeguard"] == st["n_failed"]
    res = o.cell_results(0)
    assert np.all(res["status"][res["status"] != 0] & 4)


def test_deterministic():
    mu, nu, cfg = datagen.config1_pair()
    outs = []
    for _ in range(2):
        o = ddo.Oracle(mu, nu, s=4, n_levels=1, eps=cfg["stages"][0][1], n_threads=3)
        for ell in range(4):
            o.half_iterate(ell % 2)
        outs.append(o.export())
    for k in ("row_ptr", "col", "val", "alpha_a", "alpha_b"):
        assert np.array_equal(outs[0][k], outs[1][k])


def test_invalid_inputs_rejected():
    mu, nu = datagen.small_pair(32, 3, seed=5)
    with pytest.raises(ValueError):
        ddo.Oracle(mu, nu * 2, s=4)
    bad = mu.copy()
    bad[0, 0] = -1e-3
    with pytest.raises(ValueError):
        ddo.Oracle(bad / bad.sum(), nu, s=4)
    with pytest.raises(ValueError):
        ddo.Oracle(mu[:, :30] / mu[:, :30].sum(), nu[:, :30] / nu[:, :30].sum(), s=4)


def test_accelerated_sinkhorn_same_fixed_point_fewer_loops():
    # Chebyshev-accelerated X-iteration: same stopping test, same cell optima,
    # fewer loops (compare one sweep of every cell, tight tolerance)
    mu, nu = datagen.small_pair(32, 4, seed=71)
    eps = 2.0 / 32 ** 2
    res = {}
    for accel in (0, 1):
        o = ddo.Oracle(mu, nu, s=4, n_levels=1, eps=eps, err_tol=1e-11, trunc=0.0, accel=accel,
                       newton_after=0)
        st = o.half_iterate(0)
        res[accel] = (st, o.basic_marginals())
    assert res[1][0]["loops_total"] < 0.6 * res[0][0]["loops_total"]
    assert np.abs(res[1][1] - res[0][1]).max() < 1e-9 * res[0][1].max()
    assert abs(res[1][0]["cost"] - res[0][0]["cost"]) < 1e-10


def _two_strip_cell():
    # 8x8 X block with mass only in columns 0-1 (0.55) and 6-7 (0.45); Y in two
    # 8x3 strips around them with the masses swapped (0.45 / 0.55), so exactly
    # 0.1 must cross the 4-column gap: the coupling graph of the cell is nearly
    # disconnected and plain Sinkhorn converges slowly.
    xr, xc = np.divmod(np.arange(64), 8)
    mu = np.where((xc < 2) | (xc >= 6), 1.0, 0.0) * (1 + 0.1 * np.sin(np.arange(64)))
    mu[xc < 2] *= 0.55 / mu[xc < 2].sum()
    mu[xc >= 6] *= 0.45 / mu[xc >= 6].sum()
    yr, yc = np.meshgrid(np.arange(1, 9), np.r_[-1, 0, 1, 6, 7, 8], indexing="ij")
    yr, yc = yr.ravel(), yc.ravel()
    nu = 1 + 0.2 * np.cos(np.arange(len(yr)))
    nu[yc < 3] *= 0.45 / nu[yc < 3].sum()
    nu[yc >= 3] *= 0.55 / nu[yc >= 3].sum()
    return xr, xc, mu, yr, yc, nu


def test_newton_fallback_on_nearly_disconnected_cell():
    xr, xc, mu, yr, yc, nu = _two_strip_cell()
    lam = 3.0
    plain = ddo.cell_solve(xr, xc, mu, yr, yc, nu, lam, 1e-12, 200000)
    newt = ddo.cell_solve(xr, xc, mu, yr, yc, nu, lam, 1e-12, 200000, newton_after=16)
    assert plain["rc"] == 0 and newt["rc"] == 0 and newt["newton"] and not plain["newton"]
    assert newt["loops"] < plain["loops"] / 10
    P = newt["plan"]
    # the plan has the Gibbs form by construction; with both marginals met it is
    # the unique entropic optimum, hence equal to the plain Sinkhorn plan
    assert np.abs(P.sum(1) - mu).sum() <= 1e-12
    assert np.abs(P.sum(0) - nu).max() < 1e-15
    assert np.abs(P - plain["plan"]).max() < 1e-12
    # mass conservation fixes what crosses the gap: 0.55 - 0.45 from left to right
    assert abs(P[xc < 2][:, yc >= 3].sum() - 0.1) < 1e-11
    assert P[xc >= 6][:, yc < 3].sum() < 1e-30


def test_newton_fallback_same_cell_optima_in_a_sweep():
    # one sweep of every cell with and without the Newton fallback (after 4
    # loops): same stopping test, so the same cell optima within tolerance
    mu, nu = datagen.small_pair(32, 4, seed=72)
    eps = 2.0 / 32 ** 2
    res = {}
    for k in (0, 4):
        o = ddo.Oracle(mu, nu, s=4, n_levels=1, eps=eps, err_tol=1e-11, trunc=0.0, accel=0,
                       newton_after=k)
        st = o.half_iterate(0)
        res[k] = (st, o.basic_marginals(), o.cell_results(0))
    assert res[0][0]["n_newton"] == 0 and res[4][0]["n_newton"] > 0
    assert res[4][0]["n_failed"] == 0
    assert (res[4][2]["status"] & 16).sum() > 0
    assert res[4][0]["loops_total"] < 0.5 * res[0][0]["loops_total"]
    assert np.abs(res[4][1] - res[0][1]).max() < 1e-9 * res[0][1].max()
    assert abs(res[4][0]["cost"] - res[0][0]["cost"]) < 1e-10


@pytest.mark.parametrize("cost_p", [2.0, 1.5, 3.0])
def test_small_eps_limit_is_the_monotone_rearrangement(cost_p):
    # 8 x N images whose rows all carry the same profile, mu = U(rows) (x) a,
    # nu = U(rows) (x) b: with c = |x-y|^2 the optimal plan keeps every row
    # and moves mass along it monotonically, so the unregularised W2^2 is the
    # one of the 1D profiles (north-west corner rule on the sorted CDFs).  As
    # eps falls through the schedule the DD cost must approach that closed
    # form monotonically, down to the discrete optimum once eps << h^p.  The
    # monotone plan is optimal for every strictly convex h(x - y) (Sec. 7.1,
    # Sec. 5), so the same holds for c = |x-y|^p, p = 1.5 and 3.
    N, H = 32, 8
    c = np.arange(N)
    a = np.exp(-((c - 10) / 4.0) ** 2) + 0.3 * np.exp(-((c - 24) / 3.0) ** 2) + 0.02
    b = np.exp(-((c - 18) / 5.0) ** 2) + 0.02
    a /= a.sum()
    b /= b.sum()
    mu, nu = np.tile(a / H, (H, 1)), np.tile(b / H, (H, 1))
    h = 1.0 / N
    w = dense.monotone_w2sq((c + 0.5) * h, a, (c + 0.5) * h, b, p=cost_p)
    hp = h ** cost_p
    # (the oracle's accelerated cell solver: the same stopping test and fixed
    # point; the plain one needs ~1e6 loops at the last eps, where the cells
    # are nearly disconnected)
    o = ddo.Oracle(mu, nu, s=4, n_levels=1, eps=4 * hp, err_tol=1e-9, trunc=0.0,
                   n_threads=2, cost_p=cost_p)
    gaps = []
    for f in (4.0, 1.0, 0.25, 1.0 / 16, 1.0 / 64):
        o.set_eps(f * hp)
        for k in range(10):
            st = o.half_iterate(k % 2)
        gaps.append((st["cost"] - w) / w)
    # the entropic blur shrinks with eps (down to a plateau of the outer
    # iteration near 1e-6 for p != 2, where ten half-iterations per stage
    # leave the cell plans of tiny eps slightly apart)
    assert all(gaps[i + 1] < gaps[i] for i in range(3)), gaps
    assert gaps[0] > 100 * abs(gaps[-1]) and abs(gaps[-1]) < 1e-5, gaps


def test_safeguard_reaches_the_same_cell_optimum():
    # Sec. 7.4 safeguard: a cell that hits the loop cap is solved again at
    # 2 eps from its stored potential, then at eps from that solution.  With
    # a cap of 160 loops four cells of the first config-1 sweep go through
    # it; each must reach the unique cell optimum (Proposition "Optimal
    # entropic transport couplings" (i)) of the uncapped plain solve within
    # the stopping tolerance.
    mu, nu, cfg = datagen.config1_pair()
    eps = cfg["stages"][0][1]
    kw = dict(s=4, n_levels=1, eps=eps, accel=0, newton_after=0, n_threads=2)
    ref = ddo.Oracle(mu, nu, **kw)
    ref.half_iterate(0)
    rr = ref.cell_results(0)
    o = ddo.Oracle(mu, nu, max_iter=160, **kw)
    st = o.half_iterate(0)
    r = o.cell_results(0)
    sg = (r["status"] & 4) != 0
    assert st["n_safeguard"] == sg.sum() > 0 and st["n_failed"] == 0
    assert rr["loops"][sg].min() > 160  # the cap forced them through the detour
    m_cell = np.array([mu.reshape(4, 8, 4, 8)[i // 4, :, i % 4, :].sum() for i in range(16)])
    assert np.all(r["err_x"][sg] <= 1e-5 * m_cell[sg])
    assert np.all(np.abs(r["cost"][sg] - rr["cost"][sg]) <= 1e-5 * rr["cost"][sg])
    # cells that did not need it ran the same solve
    assert np.array_equal(r["loops"][~sg], rr["loops"][~sg])


def test_multiscale_schedule_ends_at_the_entropic_optimum():
    # two levels (8x8 -> 16x16), eps 1 -> (1/16)^2, then 60 more
    # half-iterations at the final eps, tight tolerance and no truncation:
    # the end state is the full-grid entropic optimum (the DD fixed point,
    # Thm. "Linear convergence"), computed here by the dense Newton solver
    N, s = 16, 4
    mu, nu = datagen.small_pair(N, 3, seed=41)
    stages = datagen.eps_schedule(N, 2)
    stages = stages[:-1] + [(stages[-1][0], stages[-1][1], stages[-1][2] + 60)]
    o = ddo.Oracle(mu, nu, s=s, n_levels=2, eps=stages[0][1], err_tol=1e-11, trunc=0.0,
                   max_iter=200000, accel=0, newton_after=0, n_threads=2)
    st = o.run_schedule(stages)
    eps = stages[-1][1]
    C = dense.grid_cost(N, N, 1.0 / N)
    P = dense.entropic_ot_newton(C, mu.ravel(), nu.ravel(), eps)[2]
    basic, _, _ = dense.grid_partitions(N, N, s)
    assert o.level_info()["level"] == 1 and st["n_failed"] == 0
    assert np.abs(o.basic_marginals() - _basic_marg_dense(P, basic)).max() < 1e-8
    # the cost of a plan whose X-marginal is off by Err = 1e-11 can move by
    # Err * max c, 2e-11 here: 1e-8 relative to the cost of 0.03
    assert abs(o.cost()["cost"] - (C * P).sum()) < 1e-8 * (C * P).sum()
