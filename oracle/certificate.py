"""FP64 primal-dual certificate of a domain-decomposition iterate (test
infrastructure only: tests, the smoke check and the bench's CPU leg use it;
the product path never does).

Follows Sec. 6.3 "Estimating the primal-dual gap" and the relative PD gap of
Sec. 7.3 (eq. RelPDGap), with the dual objective J of eq.
EntropicOTDualObjective:

    J(u, v) = int log u dmu + int log v dnu - int u (x) v dK + |K|,
    K = exp(-c/eps) mu (x) nu.

Potentials are carried in the additive form alpha = eps log u, beta = eps log v.

Steps, in the paper's order:

1. Edge weights of the A-cell graph.  Two A-cells J1, J2 are joined through
   every B-cell J_B that meets both; the oriented weight is
   q(J1, J2) = mean_{J1 n J_B} (u_A / u_B) dmu * mean_{J2 n J_B} (u_B / u_A) dmu.
2. Discrete Helmholtz step: V on the A-cells minimising the squared misfit
   between the graph gradient of V and log q over all oriented edges.
   READING: the misfit is taken as V(J2) - V(J1) - log q(J1, J2), the
   orientation under which the path product of the q's (the construction
   the least-squares step replaces) glues consistent potentials; the printed
   form has the two vertices the other way round, which would glue with
   exp(-V).  V is fixed to mean zero (the minimiser is unique up to a
   constant on a connected graph).
3. Glued X-scaling u_hat = exp(V_J) u_{A,J} on each A-cell J.
4. READING for the Y-side: instead of gluing the truncated v_J, v_hat is the
   exact Y-iteration of u_hat (the maximiser of J over v for fixed u_hat,
   Remark "Sinkhorn algorithm"), so J(u_hat, v_hat) >= J(u_hat, any glued v).
   After it, int u_hat (x) v_hat dK = |nu| = 1.
5. Relative PD gap (KL(pi|K) - J) / (KL(pi|K) - |K|); the primal score
   KL(pi|K) - |K| of the DD plan is the sum of the composite-cell objectives
   (Sec. 6.3: summed over the cells of the last half-iteration).

Parity pinned by: weak and strong duality against the dense entropic optimum,
exact recovery of a planted gradient by the Helmholtz step, and the gap of a
converged DD iterate tending to zero (tests/test_certificate.py).
"""
import numpy as np
from scipy.special import logsumexp


def dual_objective(alpha, beta, C, mu, nu, eps):
    """J(u, v) - |K| of eq. EntropicOTDualObjective written out densely
    (u = exp(alpha/eps), v = exp(beta/eps), K = exp(-c/eps) mu nu)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    mass = np.sum(np.exp((alpha[:, None] + beta[None, :] - C) / eps) * np.outer(mu, nu))
    return float(np.dot(alpha, mu) / eps + np.dot(beta, nu) / eps - mass)


def primal_score(plan, C, mu, nu, eps):
    """KL(pi|K) - |K| = sum pi log(pi/K) - |pi| (Definition "Kullback-Leibler divergence")."""
    P = np.asarray(plan, dtype=np.float64)
    logK = -C / eps + np.log(mu)[:, None] + np.log(nu)[None, :]  # log form: K underflows at small eps
    pos = P > 0
    return float(np.sum(P[pos] * (np.log(P[pos]) - logK[pos])) - P.sum())


def graph_edges(alpha_a, alpha_b, mu, eps, basic, cells_a, cells_b):
    """Oriented edges (J1, J2, log q(J1, J2)) of the A-cell graph (step 1).

    basic: pixel index arrays of the basic cells; cells_a / cells_b: lists of
    basic-cell ids of the composite cells.  The means are mu-weighted averages
    over J1 n J_B and J2 n J_B, evaluated with a max shift for range."""
    a_of_basic = {}
    for J, cell in enumerate(cells_a):
        for i in cell:
            a_of_basic[i] = J
    edges = []
    for cell_b in cells_b:
        pix_by_a = {}
        for i in cell_b:
            pix_by_a.setdefault(a_of_basic[i], []).append(basic[i])
        parts = {J: np.concatenate(p) for J, p in pix_by_a.items()}
        lmean_ab, lmean_ba = {}, {}
        for J, xs in parts.items():
            with np.errstate(divide="ignore"):  # pixels without mass: weight e^-inf = 0
                w = np.log(mu[xs]) - np.log(mu[xs].sum())
            d = (alpha_a[xs] - alpha_b[xs]) / eps
            lmean_ab[J] = logsumexp(d + w)
            lmean_ba[J] = logsumexp(-d + w)
        for J1 in parts:
            for J2 in parts:
                if J1 != J2:
                    edges.append((J1, J2, lmean_ab[J1] + lmean_ba[J2]))
    return edges


def helmholtz(edges, n_cells):
    """Mean-zero V minimising sum_e (V(J2) - V(J1) - log q_e)^2 (step 2)."""
    if not edges:
        return np.zeros(n_cells)
    D = np.zeros((len(edges), n_cells))
    w = np.empty(len(edges))
    for e, (J1, J2, lq) in enumerate(edges):
        D[e, J2] += 1.0
        D[e, J1] -= 1.0
        w[e] = lq
    V = np.linalg.lstsq(D, w, rcond=None)[0]
    return V - V.mean()


def helmholtz_sparse(edges, n_cells):
    """The same minimiser as `helmholtz` for large graphs: the normal
    equations L V = D^T w (L the graph Laplacian) with V(0) = 0, solved by a
    sparse direct factorisation, then shifted to mean zero."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    if not edges or n_cells == 1:
        return np.zeros(n_cells)
    e = np.array([(a, b) for a, b, _ in edges], dtype=np.int64)
    w = np.array([lq for _, _, lq in edges])
    ne = len(edges)
    D = sp.csr_matrix((np.concatenate([-np.ones(ne), np.ones(ne)]),
                       (np.concatenate([np.arange(ne)] * 2), np.concatenate([e[:, 0], e[:, 1]]))),
                      shape=(ne, n_cells))
    L = (D.T @ D).tocsc()
    rhs = D.T @ w
    V = np.zeros(n_cells)
    V[1:] = spl.spsolve(L[1:, 1:], rhs[1:])
    return V - V.mean()


def y_iteration(alpha, C, mu, eps, chunk=2048, support=None):
    """beta(y) = -eps log sum_x exp((alpha(x) - c(x,y))/eps) mu(x) (step 4);
    with a boolean support matrix the sum runs over its True entries only
    (the stored support of a truncated plan)."""
    with np.errstate(divide="ignore"):  # log 0 = -inf: pixels without mass drop out
        lmu = np.log(mu)
    out = np.empty(C.shape[1])
    for j0 in range(0, C.shape[1], chunk):
        t = (alpha[:, None] - C[:, j0:j0 + chunk]) / eps + lmu[:, None]
        if support is not None:
            t = np.where(support[:, j0:j0 + chunk], t, -np.inf)
        out[j0:j0 + chunk] = -eps * logsumexp(t, axis=0)
    return out


def plan_support(row_ptr, col, basic, n_px):
    """Boolean (x, y) mask of the pairs a basic-cell CSR stores: X_i x supp(nu_i)."""
    S = np.zeros((n_px, n_px), dtype=bool)
    for i, xs in enumerate(basic):
        S[np.ix_(xs, col[row_ptr[i]:row_ptr[i + 1]])] = True
    return S


def certificate(alpha_a, alpha_b, obj, C, mu, nu, eps, basic, cells_a, cells_b, support=None):
    """Glued dual candidate and relative PD gap of a DD iterate (steps 1-5).

    alpha_a, alpha_b: the stored X-potentials of the two partitions (per pixel,
    any constant per composite cell); obj: eps * (KL(pi|K) - |K|) of the
    primal iterate; support: optional mask restricting the Y-iteration.  Returns a dict with V, the glued alpha_hat, beta_hat,
    J - |K| and the relative gap."""
    alpha_a = np.asarray(alpha_a, dtype=np.float64).ravel()
    alpha_b = np.asarray(alpha_b, dtype=np.float64).ravel()
    edges = graph_edges(alpha_a, alpha_b, mu, eps, basic, cells_a, cells_b)
    V = helmholtz(edges, len(cells_a))
    alpha_hat = alpha_a.copy()
    for J, cell in enumerate(cells_a):
        for i in cell:
            alpha_hat[basic[i]] += eps * V[J]
    beta_hat = y_iteration(alpha_hat, C, mu, eps, support=support)
    # <alpha, mu> and <beta, nu> are integrals against the marginals: pixels
    # of zero mass contribute nothing (there beta_hat may be infinite, when no
    # stored pair reaches the pixel)
    xm, ym = mu > 0, nu > 0
    dual = float(np.dot(alpha_hat[xm], mu[xm]) / eps + np.dot(beta_hat[ym], nu[ym]) / eps
                 - nu.sum())
    primal = obj / eps
    return {"V": V, "alpha_hat": alpha_hat, "beta_hat": beta_hat, "dual": dual,
            "primal": primal, "gap": primal - dual, "rel_gap": (primal - dual) / primal,
            "n_edges": len(edges)}
