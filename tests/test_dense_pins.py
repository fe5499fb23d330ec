"""Pins of the dense FP64 references against what the paper and the mathematics fix.

Nothing here compares a reference with a retyped copy of itself: each test
uses a closed form, a brute-force minimisation, an exact identity from the
paper, or a textbook algorithm (odd-even transposition sort).
"""
import json
import os

import numpy as np
import pytest
from scipy.optimize import minimize, minimize_scalar

from oracle import dense

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand_problem(nx, ny, seed):
    rng = np.random.default_rng(seed)
    C = rng.uniform(0, 1, size=(nx, ny))
    mu = rng.uniform(0.2, 1, nx)
    nu = rng.uniform(0.2, 1, ny)
    return C, mu / mu.sum(), nu / nu.sum()


def test_single_source_point_plan_is_nu():
    # with one X point the only coupling is pi(x0, .) = nu
    C, _, nu = _rand_problem(1, 7, 0)
    f, g, p, it, err = dense.sinkhorn(C, np.array([1.0]), nu, 0.05, tol=1e-13)
    assert np.allclose(p[0], nu, rtol=0, atol=1e-15)


def test_newton_and_sinkhorn_agree():
    # two independent solvers of the same strictly convex problem
    C, mu, nu = _rand_problem(7, 9, 9)
    for eps in (0.3, 0.03):
        p1 = dense.entropic_ot_newton(C, mu, nu, eps)[2]
        p2 = dense.sinkhorn(C, mu, nu, eps, tol=1e-13)[2]
        assert np.abs(p1 - p2).max() < 1e-12


def test_large_eps_gives_product():
    # as eps -> infinity the entropic optimum tends to mu x nu
    C, mu, nu = _rand_problem(5, 6, 1)
    p = dense.entropic_ot(C, mu, nu, 1e7)
    assert np.abs(p - np.outer(mu, nu)).max() < 1e-7


def test_two_by_two_brute_force():
    # Pi(mu,nu) for 2x2 is one-dimensional: pi = [[a, m0-a],[n0-a, 1-m0-n0+a]]
    C, mu, nu = _rand_problem(2, 2, 2)
    eps = 0.1
    K = dense.kernel(C, mu, nu, eps)

    def obj(a):
        pi = np.array([[a, mu[0] - a], [nu[0] - a, 1 - mu[0] - nu[0] + a]])
        return eps * dense.kl(pi, K) if np.all(pi >= 0) else np.inf

    lo = max(0.0, mu[0] + nu[0] - 1)
    hi = min(mu[0], nu[0])
    r = minimize_scalar(obj, bounds=(lo, hi), method="bounded",
                        options={"xatol": 1e-14})
    p = dense.entropic_ot(C, mu, nu, eps)
    assert abs(p[0, 0] - r.x) < 1e-8


def test_three_by_three_brute_force():
    # free parameters: the upper-left 2x2 block; the rest follows from the marginals
    C, mu, nu = _rand_problem(3, 3, 3)
    eps = 0.2
    K = dense.kernel(C, mu, nu, eps)

    def plan(z):
        a = z.reshape(2, 2)
        pi = np.zeros((3, 3))
        pi[:2, :2] = a
        pi[:2, 2] = mu[:2] - a.sum(1)
        pi[2, :2] = nu[:2] - a.sum(0)
        pi[2, 2] = 1 - pi[:2, :].sum() - pi[2, :2].sum()
        return pi

    def obj(z):
        pi = plan(z)
        if np.any(pi <= 0):
            return 1e9
        return eps * dense.kl(pi, K)

    z0 = np.outer(mu, nu)[:2, :2].ravel()
    r = minimize(obj, z0, method="Nelder-Mead",
                 options={"xatol": 1e-13, "fatol": 1e-16, "maxiter": 20000, "maxfev": 40000})
    p = dense.entropic_ot(C, mu, nu, eps)
    assert np.abs(plan(r.x) - p).max() < 1e-7


def test_duality_gap_closes():
    # Proposition "Duality": J(u,v) <= KL(pi|K), equality for the scaling-form optimum
    C, mu, nu = _rand_problem(6, 5, 4)
    eps = 0.07
    f, g, p, it, err = dense.sinkhorn(C, mu, nu, eps, tol=1e-13)
    K = dense.kernel(C, mu, nu, eps)
    J = np.sum(mu * f / eps) + np.sum(nu * g / eps) - p.sum() + K.sum()
    primal = dense.kl(p, K)
    assert J <= primal + 1e-12
    assert primal - J < 1e-10
    # and a perturbed dual is strictly worse
    J2 = np.sum(mu * (f / eps + 0.1)) + np.sum(nu * g / eps) - np.exp(0.1) * p.sum() + K.sum()
    assert J2 < J


def test_marginals_after_y_iteration():
    C, mu, nu = _rand_problem(9, 11, 5)
    f, g, p, it, err = dense.sinkhorn(C, mu, nu, 0.02, tol=1e-6)
    assert np.allclose(p.sum(0), nu, rtol=1e-13, atol=0)  # Y-marginal exact
    assert np.abs(p.sum(1) - mu).sum() <= 1e-6 * mu.sum() + 1e-15
    assert abs(err - np.abs(p.sum(1) - mu).sum()) < 1e-14


def test_monotone_rearrangement_closed_form():
    # two-point example done by hand: W2^2 of 1/2(d0+d1) -> 1/2(d1+d3) = 1/2(1 + 4) = 2.5
    assert abs(dense.monotone_w2sq([0, 1], [0.5, 0.5], [3, 1], [0.5, 0.5]) - 2.5) < 1e-15


def test_1d_small_eps_approaches_monotone_rearrangement():
    # 1D, c = |x-y|^2: as eps -> 0 the entropic cost tends to the monotone W2^2
    n = 24
    rng = np.random.default_rng(6)
    x = np.sort(rng.uniform(0, 1, n))
    y = np.sort(rng.uniform(0, 1, n)) * 0.7 + 0.2
    a = rng.uniform(0.5, 1, n)
    b = rng.uniform(0.5, 1, n)
    a /= a.sum()
    b /= b.sum()
    C = (x[:, None] - y[None, :]) ** 2
    w = dense.monotone_w2sq(x, a, y, b)
    gaps = []
    for eps in [1e-2, 3e-3, 1e-3, 3e-4]:
        p = dense.sinkhorn(C, a, b, eps, tol=1e-12, max_iter=400000)[2]
        gaps.append(abs((C * p).sum() - w))
    assert all(gaps[i + 1] < gaps[i] for i in range(len(gaps) - 1))
    assert gaps[-1] < 4e-3 * w


def _three_cell(eps, q=0.3, n_half=30):
    d = json.load(open(os.path.join(GOLD, "worst_case_three.json")))
    C = np.array(d["cost"], dtype=float)
    p = (1 - q) / 2
    mu = np.array([p, q, p])
    sub = {"0": 0.0, "p": p, "q": q}
    pi0 = np.array([[sub[v] for v in row] for row in d["pi0_pattern"]])
    basic = [np.array([0]), np.array([1]), np.array([2])]
    plans = dense.dd_dense(C, mu, mu, eps, d["cells_a"], d["cells_b"], basic, pi0, n_half,
                           tol=1e-13)
    pistar = dense.entropic_ot(C, mu, mu, eps)
    return C, mu, pi0, plans, pistar


@pytest.mark.parametrize("eps", [2.0, 3.0, 5.0, 10.0])
def test_three_cell_rate_bound(eps):
    C, mu, pi0, plans, pistar = _three_cell(eps)
    q = 0.3
    lam = 1.0 / (1.0 + np.exp(-2 * 10.0 / eps) * q / (1 - q))
    K = dense.kernel(C, mu, mu, eps)
    kl_star = dense.kl(pistar, K)
    delta = [dense.kl(p, K) - kl_star for p in plans]
    checked = 0
    for ell in range(2, len(plans)):
        if delta[ell - 1] < 1e-11:
            break
        assert delta[ell] <= lam * delta[ell - 1] + 1e-13
        checked += 1
    assert checked >= 3
    # every iterate is feasible (Proposition after Algorithm 1)
    for p in plans[1:]:
        assert np.allclose(p.sum(1), mu, atol=1e-12) and np.allclose(p.sum(0), mu, atol=1e-12)


@pytest.mark.parametrize("eps", [3.0, 10.0])
def test_suboptimality_identities(eps):
    # Lemma "Expressions for decrement and sub-optimality"
    C, mu, pi0, plans, pistar = _three_cell(eps, n_half=8)
    K = dense.kernel(C, mu, mu, eps)
    kl_star = dense.kl(pistar, K)
    for ell in range(2, len(plans)):
        d_prev = dense.kl(plans[ell - 1], K) - kl_star
        d_cur = dense.kl(plans[ell], K) - kl_star
        assert abs((d_prev - d_cur) - dense.kl(plans[ell - 1], plans[ell])) < 1e-10
        assert abs(d_cur - dense.kl(plans[ell], pistar)) < 1e-10


def _chain(N, n_half):
    C = np.full((N, N), 10.0)
    np.fill_diagonal(C, 0.0)
    C[0, N - 1] = C[N - 1, 0] = 1.0
    mu = np.full(N, 1.0 / N)
    pi0 = np.eye(N) / N
    pi0[0, 0] = pi0[N - 1, N - 1] = 0.0
    pi0[0, N - 1] = pi0[N - 1, 0] = 1.0 / N
    basic = [np.array([i]) for i in range(N)]
    cells_a = [[i, i + 1] for i in range(0, N - 1, 2)] + ([[N - 1]] if N % 2 else [])
    cells_b = [[0]] + [[i, i + 1] for i in range(1, N - 1, 2)] + ([[N - 1]] if N % 2 == 0 else [])
    eps = 1.4
    plans = dense.dd_dense(C, mu, mu, eps, cells_a, cells_b, basic, pi0, n_half, tol=1e-13)
    K = dense.kernel(C, mu, mu, eps)
    ks = dense.kl(dense.entropic_ot(C, mu, mu, eps), K)
    return np.array([dense.kl(p, K) - ks for p in plans])


def test_chain_golden_setup_matches():
    d = json.load(open(os.path.join(GOLD, "chain.json")))
    N = 5
    C = np.full((N, N), 10.0)
    np.fill_diagonal(C, 0.0)
    C[0, N - 1] = C[N - 1, 0] = 1.0
    assert np.array_equal(C, np.array(d["cost_N5"], dtype=float))


def test_chain_contraction_slows_with_length():
    # Example "Chain graph": the empirical contraction factor approaches 1 as N grows
    lams = []
    for N in (4, 6, 8):
        d = _chain(N, 60)
        tail = d[20:60]
        tail = tail[tail > 1e-13]
        lam = np.exp(np.polyfit(np.arange(len(tail)), np.log(tail), 1)[0])
        lams.append(lam)
    assert lams[0] < lams[1] < lams[2] < 1.0


def test_odd_even_transposition_sort_limit():
    # Sec. 5: singleton basic cells, pairs as composite cells, strictly Monge
    # cost, tiny eps: each DD iteration is one phase of odd-even transposition sort
    N = 8
    rng = np.random.default_rng(8)
    perm = rng.permutation(N)
    x = np.arange(N, dtype=float)
    C = (x[:, None] - x[None, :]) ** 2
    mu = np.full(N, 1.0 / N)
    pi0 = np.zeros((N, N))
    pi0[np.arange(N), perm] = 1.0 / N
    basic = [np.array([i]) for i in range(N)]
    cells_a = [[i, i + 1] for i in range(0, N, 2)]
    cells_b = [[0]] + [[i, i + 1] for i in range(1, N - 1, 2)] + [[N - 1]]
    plans = dense.dd_dense(C, mu, mu, 0.25, cells_a, cells_b, basic, pi0, N, tol=1e-12)
    state = perm.copy()
    for ell in range(1, N + 1):
        start = 0 if ell % 2 == 1 else 1
        for i in range(start, N - 1, 2):
            if state[i] > state[i + 1]:
                state[i], state[i + 1] = state[i + 1], state[i]
        assign = plans[ell].argmax(axis=1)
        assert np.array_equal(assign, state), ell
        assert plans[ell].max(axis=1).min() > (1.0 / N) * 0.95
    assert np.array_equal(state, np.arange(N))
