"""Pins of the FP64 primal-dual certificate (CPU only): duality facts of
Proposition "Duality for regularized optimal transport", exact recovery of a
planted gradient by the Helmholtz step, and the gap of a converged DD iterate."""
import numpy as np

from oracle import certificate as cert
from oracle import dense, ddo
from paper_2001_10986_amd import datagen


def _pair(N, seed):
    mu, nu = datagen.small_pair(N, 3, seed=seed)
    return mu.ravel(), nu.ravel()


def test_strong_and_weak_duality():
    N = 8
    mu, nu = _pair(N, 3)
    eps = 4.0 / N ** 2
    C = dense.grid_cost(N, N, 1.0 / N)
    f, g, P, _, _ = dense.sinkhorn(C, mu, nu, eps, tol=1e-14)
    primal = cert.primal_score(P, C, mu, nu, eps)
    # strong duality at the optimum: J(u*, v*) = KL(pi*|K)
    assert abs(cert.dual_objective(f, g, C, mu, nu, eps) - primal) < 1e-9 * abs(primal)
    # weak duality for arbitrary scalings against two feasible plans
    rng = np.random.default_rng(0)
    prod = cert.primal_score(np.outer(mu, nu), C, mu, nu, eps)
    for _ in range(5):
        a = f + eps * rng.normal(0, 0.5, f.shape)
        b = g + eps * rng.normal(0, 0.5, g.shape)
        J = cert.dual_objective(a, b, C, mu, nu, eps)
        assert J <= primal + 1e-9 and J <= prod + 1e-9
    # the exact Y-iteration is the maximiser over v: it cannot lower J
    a = f + eps * rng.normal(0, 0.5, f.shape)
    b = cert.y_iteration(a, C, mu, eps)
    J_best = cert.dual_objective(a, b, C, mu, nu, eps)
    for _ in range(5):
        assert cert.dual_objective(a, b + eps * rng.normal(0, 0.3, b.shape), C, mu, nu, eps) <= J_best
    # and after it the kernel mass is |nu|, the shortcut used by the certificate
    mass = np.sum(np.exp((a[:, None] + b[None, :] - C) / eps) * np.outer(mu, nu))
    assert abs(mass - nu.sum()) < 1e-13


def test_helmholtz_recovers_planted_gradient():
    # consistent potentials: alpha_A = phi - eps*V(A(x)), alpha_B = phi + eps*c(B(x))
    N, s = 32, 4
    mu, _ = _pair(N, 5)
    eps = 1e-3
    basic, ca, cb = dense.grid_partitions(N, N, s)
    rng = np.random.default_rng(2)
    phi = rng.normal(0, 1e-2, N * N)
    V_true = rng.normal(0, 3, len(ca))
    V_true -= V_true.mean()
    cB = rng.normal(0, 3, len(cb))
    aA, aB = phi.copy(), phi.copy()
    for J, cell in enumerate(ca):
        for i in cell:
            aA[basic[i]] -= eps * V_true[J]
    for J, cell in enumerate(cb):
        for i in cell:
            aB[basic[i]] += eps * cB[J]
    edges = cert.graph_edges(aA, aB, mu, eps, basic, ca, cb)
    # every B-cell meeting k A-cells gives k(k-1) oriented edges
    assert len(edges) == sum(len(c) * (len(c) - 1) for c in cb)
    V = cert.helmholtz(edges, len(ca))
    assert np.abs(V - V_true).max() < 1e-9
    # the glued potential is phi up to one constant
    glued = aA.copy()
    for J, cell in enumerate(ca):
        for i in cell:
            glued[basic[i]] += eps * V[J]
    d = glued - phi
    assert np.ptp(d) < 1e-12


def _run_dd(N, s, eps, n_half, seed=11):
    mu, nu = datagen.small_pair(N, 3, seed=seed)
    o = ddo.Oracle(mu, nu, s=s, n_levels=1, eps=eps, err_tol=1e-10, trunc=0.0, max_iter=200000)
    for ell in range(n_half):
        o.half_iterate(ell % 2)
    e = o.export()
    return mu.ravel(), nu.ravel(), e, o.cost()["obj"]


def test_gap_vanishes_at_the_optimum_whatever_the_cell_constants():
    # DD started from the entropic optimum (its basic-cell marginals and
    # potential) stays there; the certificate must then close the gap, also
    # after arbitrary constants are added to the potentials cell by cell
    # (the gauge freedom of each composite problem that the gluing removes)
    N, s = 16, 4
    eps = 4.0 / N ** 2
    C = dense.grid_cost(N, N, 1.0 / N)
    basic, ca, cb = dense.grid_partitions(N, N, s)
    mu, nu = datagen.small_pair(N, 3, seed=11)
    m, n = mu.ravel(), nu.ravel()
    f, g, P, _, _ = dense.sinkhorn(C, m, n, eps, tol=1e-14)
    opt = cert.primal_score(P, C, m, n, eps)
    rp, col, val = [0], [], []
    for xs in basic:
        v = P[xs, :].sum(0)
        nz = np.nonzero(v > 0)[0]
        col += list(nz)
        val += list(v[nz])
        rp.append(len(col))
    o = ddo.Oracle(mu, nu, s=s, n_levels=1, eps=eps, err_tol=1e-12, trunc=0.0)
    o.import_state(0, eps, np.array(rp), np.array(col), np.array(val), f.reshape(N, N),
                   f.reshape(N, N))
    o.half_iterate(0)
    o.half_iterate(1)
    e = o.export()
    obj = o.cost()["obj"]
    assert abs(obj / eps - opt) < 1e-10 * opt
    rng = np.random.default_rng(9)
    aA, aB = e["alpha_a"].ravel().copy(), e["alpha_b"].ravel().copy()
    for cells, a in ((ca, aA), (cb, aB)):
        for cell in cells:
            sh = eps * rng.normal(0, 5)
            for i in cell:
                a[basic[i]] += sh
    for A, B in ((e["alpha_a"], e["alpha_b"]), (aA, aB)):
        r = cert.certificate(A, B, obj, C, m, n, eps, basic, ca, cb)
        assert abs(r["rel_gap"]) < 1e-11
        assert abs(r["dual"] - opt) < 1e-10 * opt
        # the certificate's dual value is J of the glued pair written out densely
        J = cert.dual_objective(r["alpha_hat"], r["beta_hat"], C, m, n, eps)
        assert abs(J - r["dual"]) < 1e-10 * abs(J)


def test_gap_brackets_the_optimum_before_convergence():
    N, s = 16, 4
    eps = 4.0 / N ** 2
    C = dense.grid_cost(N, N, 1.0 / N)
    basic, ca, cb = dense.grid_partitions(N, N, s)
    opt = None
    for n_half in (3, 10):
        mu, nu, e, obj = _run_dd(N, s, eps, n_half)
        if opt is None:
            opt = cert.primal_score(dense.entropic_ot(C, mu, nu, eps), C, mu, nu, eps)
        r = cert.certificate(e["alpha_a"], e["alpha_b"], obj, C, mu, nu, eps, basic, ca, cb)
        # weak duality: the glued dual value and the DD primal score bracket the optimum
        assert r["dual"] < opt < r["primal"]
        assert r["rel_gap"] > 0


def test_paper_protocol_gap_within_table_summary():
    # The paper's own protocol (Sec. 7.1: layers from 8x8, 4/2/2 half-
    # iterations at eps = 2, 1, 1/2 dx_l^2, 2 more at dx^2/4; Err 1e-4) on a
    # 64x64 blob pair, run by the plain FP64 oracle, then certified: the
    # relative PD gap must fall in the range Table "Summary" prints for that
    # size (mean 1.9e-4, std 1.6e-4 over 45 pairs; ours are other random
    # images, so the bar is the mean plus two standard deviations).  The same
    # pair run with a single 64x64 level from eps = 1 leaves a gap near 0.25:
    # the protocol, not the certificate, sets how small the gap gets.
    import json
    import os
    tab = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                      "table_summary_pd_gap.json")))
    k = tab["sizes"].index(64)
    bar = tab["rel_pd_gap_mean"][k] + 2 * tab["rel_pd_gap_std"][k]
    N = 64
    mu, nu = datagen.small_pair(N, 8, seed=11)
    stages, nlev = datagen.paper_schedule(N)
    o = ddo.Oracle(mu, nu, s=4, n_levels=nlev, eps=stages[0][1], err_tol=1e-4, accel=0,
                   newton_after=0)
    o.run_schedule(stages)
    c = o.cost()
    assert c["err_x"] <= 1e-4 and c["err_y"] <= 1e-6
    eps = stages[-1][1]
    e = o.export()
    C = dense.grid_cost(N, N, 1.0 / N)
    basic, ca, cb = dense.grid_partitions(N, N, 4)
    r = cert.certificate(e["alpha_a"], e["alpha_b"], c["obj"], C, mu.ravel(), nu.ravel(), eps,
                         basic, ca, cb)
    assert 0 < r["rel_gap"] < bar, r["rel_gap"]


def test_sparse_helmholtz_equals_dense_least_squares():
    # the sparse normal-equation solve used for large graphs gives the
    # minimiser of the dense least squares
    N, s = 32, 4
    mu, _ = _pair(N, 5)
    eps = 1e-3
    basic, ca, cb = dense.grid_partitions(N, N, s)
    rng = np.random.default_rng(4)
    aA = rng.normal(0, 1e-2, N * N)
    aB = rng.normal(0, 1e-2, N * N)
    edges = cert.graph_edges(aA, aB, mu, eps, basic, ca, cb)
    V1 = cert.helmholtz(edges, len(ca))
    V2 = cert.helmholtz_sparse(edges, len(ca))
    assert np.abs(V1 - V2).max() < 1e-10 * np.abs(V1).max()
