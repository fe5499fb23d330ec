"""Basic cells of 2 x 2 pixels (s = 2; Sec. 7.1 "Basic and composite
partitions": the cell size trades cell difficulty against the number of
cells and of iterations) on the GPU against the FP64 oracle run with the
same s.  A composite cell of 4 x 4 pixels occupies the top-left corner of the
solvers' 8 x 8 block, the rest of the block carries no mass."""
import numpy as np
import pytest

from paper_2001_10986_amd import datagen

pytestmark = pytest.mark.gpu

BARY_PX = 1e-2


def _summary(e, W):
    rp, col, val = e["row_ptr"], e["col"], e["val"]
    out = np.empty((len(rp) - 1, 3))
    for b in range(len(rp) - 1):
        v, c = val[rp[b]:rp[b + 1]], col[rp[b]:rp[b + 1]]
        m = v.sum()
        out[b] = (m, np.dot(v, c // W) / m, np.dot(v, c % W) / m)
    return out


@pytest.mark.parametrize("N", [16, 32])
def test_half_iterations_match_oracle(N):
    from oracle import ddo
    from paper_2001_10986_amd import dd
    mu, nu = datagen.small_pair(N, 3, seed=5)
    eps = 4.0 / N ** 2
    g = dd.Problem(mu, nu, [(0, eps, 4)], s=2, n_levels=1)
    o = ddo.Oracle(mu, nu, s=2, n_levels=1, eps=eps)
    info = g.level_info()
    assert info["n_basic"] == (N // 2) ** 2 and info["n_cells_a"] == (N // 4) ** 2
    for ell in range(4):
        sg = g.half_iterate(ell % 2)
        so = o.half_iterate(ell % 2)
        print(N, ell, "cost", sg["cost"], so["cost"], "loops", sg["loops_total"],
              so["loops_total"], flush=True)
        assert sg["n_failed"] == 0 and so["n_failed"] == 0
        assert abs(sg["cost"] - so["cost"]) <= 1e-7 * so["cost"]
        assert abs(sg["obj"] - so["obj"]) <= 1e-6 * abs(so["obj"])
        assert sg["err_x"] <= 1e-5
        assert abs(sg["loops_total"] - so["loops_total"]) <= 0.02 * so["loops_total"] + 2
        bg, bo = g.basic_marginals(), o.basic_marginals()
        assert np.abs(bg - bo).max() < 1e-6 * bg.sum(axis=1).max()
        # |nu_i| = |mu_i| for every 2x2 basic cell, up to the truncated mass
        m_i = mu.reshape(N // 2, 2, N // 2, 2).sum(axis=(1, 3)).ravel()
        assert np.abs(bg.sum(axis=1) - m_i).max() < 1e-15 * N * N + 1e-14


def test_multilevel_end_to_end_vs_plain_oracle():
    from oracle import ddo
    from paper_2001_10986_amd import dd
    mu, nu = datagen.small_pair(64, 4, seed=17)
    stages = datagen.eps_schedule(64, 2)
    g = dd.Problem(mu, nu, stages, s=2, n_levels=2)
    rs = g.run_schedule()
    o = ddo.Oracle(mu, nu, s=2, n_levels=2, eps=stages[0][1], accel=0, newton_after=0)
    o.run_schedule(stages)
    cg, co = g.cost(), o.cost()
    sg, so = _summary(g.export(), 64), _summary(o.export(), 64)
    d = np.abs(sg[:, 1:] - so[:, 1:]).max()
    print("s=2 cost gpu", cg["cost"], "oracle", co["cost"], "barycentres px", d, flush=True)
    assert rs["n_failed"] == 0 and cg["level"] == co["level"] == 1
    assert abs(cg["cost"] - co["cost"]) <= 1e-5 * co["cost"]
    assert cg["err_x"] <= 1e-5 and cg["err_y"] <= 1e-5
    assert np.abs(sg[:, 0] - so[:, 0]).max() <= 1e-12
    assert d <= BARY_PX


def test_refine_matches_oracle_from_same_state():
    from oracle import ddo
    from paper_2001_10986_amd import dd
    mu, nu = datagen.small_pair(64, 4, seed=23)
    eps = 2.0 ** -9
    g = dd.Problem(mu, nu, [(0, eps, 4)], s=2, n_levels=2)
    for ell in range(4):
        g.half_iterate(ell % 2)
    e = g.export()
    o = ddo.Oracle(mu, nu, s=2, n_levels=2, eps=eps)
    o.import_state(0, eps, e["row_ptr"], e["col"], e["val"], e["alpha_a"], e["alpha_b"])
    g.refine()
    o.refine()
    eg, eo = g.export(), o.export()
    assert np.array_equal(eg["row_ptr"], eo["row_ptr"])
    assert np.array_equal(eg["col"], eo["col"])
    assert np.abs(eg["val"] - eo["val"]).max() <= 1e-15 * eo["val"].max() * 4
    assert np.abs(eg["alpha_a"] - eo["alpha_a"]).max() < 1e-9 * np.abs(eo["alpha_a"]).max() + 1e-12


def test_certificate_matches_oracle():
    from oracle import certificate as cert
    from oracle import dense
    from paper_2001_10986_amd import dd
    N = 32
    mu, nu = datagen.small_pair(N, 4, seed=7)
    eps = 4.0 / N ** 2
    g = dd.Problem(mu, nu, [(0, eps, 8)], s=2, n_levels=1)
    for ell in range(8):
        g.half_iterate(ell % 2)
    r = g.certificate(potentials=True)
    e = g.export()
    C = dense.grid_cost(N, N, 1.0 / N)
    basic, ca, cb = dense.grid_partitions(N, N, 2)
    sup = cert.plan_support(e["row_ptr"], e["col"], basic, N * N)
    o = cert.certificate(e["alpha_a"], e["alpha_b"], g.cost()["obj"], C, mu.ravel(), nu.ravel(),
                         eps, basic, ca, cb, support=sup)
    scale = np.abs(o["alpha_hat"]).max()
    assert r["n_edges"] == o["n_edges"]
    assert np.abs(r["alpha_hat"].ravel() - o["alpha_hat"]).max() < 1e-10 * scale + 1e-13
    assert abs(r["rel_gap"] - o["rel_gap"]) < 1e-10 and r["rel_gap"] > 0


def test_paper_protocol_gap_with_small_cells():
    # The paper's protocol on a 64x64 pair (layers from 8x8, 4/2/2
    # half-iterations per layer, Err 1e-4) with s = 2 and s = 4.  Sec. 7.1:
    # smaller cells need more iterations, so the same number of iterations
    # leaves the iterate further from the optimum: the relative PD gap with
    # s = 2 exceeds the one with s = 4 (measured 1.2e-3 against 2.5e-4).
    # GPU and oracle agree on it for s = 2.
    from oracle import certificate as cert
    from oracle import ddo, dense
    from paper_2001_10986_amd import dd
    N = 64
    mu, nu = datagen.small_pair(N, 8, seed=11)
    stages, nlev = datagen.paper_schedule(N)
    gaps = {}
    for s in (2, 4):
        g = dd.Problem(mu, nu, stages, s=s, n_levels=nlev, err_tol=1e-4)
        rs = g.run_schedule()
        gaps[s] = (g.certificate()["rel_gap"], g.cost()["cost"], rs["n_cell_solves"])
        g.close()
    o = ddo.Oracle(mu, nu, s=2, n_levels=nlev, eps=stages[0][1], err_tol=1e-4, accel=0,
                   newton_after=0)
    o.run_schedule(stages)
    e = o.export()
    basic, ca, cb = dense.grid_partitions(N, N, 2)
    ro = cert.certificate(e["alpha_a"], e["alpha_b"], o.cost()["obj"], dense.grid_cost(N, N, 1.0 / N),
                          mu.ravel(), nu.ravel(), stages[-1][1], basic, ca, cb)
    print(f"paper protocol 64x64: rel gap s=2 gpu {gaps[2][0]:.4e} oracle {ro['rel_gap']:.4e}, "
          f"s=4 gpu {gaps[4][0]:.4e}; cell solves {gaps[2][2]} / {gaps[4][2]}", flush=True)
    assert 0 < gaps[4][0] < gaps[2][0]
    assert abs(gaps[2][0] - ro["rel_gap"]) <= 0.05 * ro["rel_gap"]
    assert abs(gaps[2][1] - o.cost()["cost"]) <= 1e-4 * o.cost()["cost"]


def test_network_features_refused():
    from paper_2001_10986_amd import dd, mlp
    mu, nu = datagen.small_pair(32, 3, seed=5)
    g = dd.Problem(mu, nu, [(0, 0.01, 2)], s=2)
    with pytest.raises(dd.DDError):
        g.set_warm_start(mlp.MLP(768, 64, 256, seed=1), 3, 0.5)
    g.close()
