"""Dense FP64 NumPy references (test infrastructure only).

These are the textbook objects the sparse C oracle is pinned to:

- ``sinkhorn``: log-domain Sinkhorn on a dense cost matrix (Remark "Sinkhorn
  algorithm"), stopping on the L1 error of the X-marginal after a
  Y-iteration, as in Sec. 6.2.
- ``entropic_ot_newton``: the same optimum by damped Newton on the dual, an
  algorithm independent of Sinkhorn.
- ``entropic_ot``: the unique entropic optimum (Proposition "Optimal entropic
  transport couplings" (i)) computed by that Sinkhorn to a tight tolerance.
- ``dd_dense``: Algorithm 1 (entropic domain decomposition) on a dense plan,
  each composite-cell problem solved to a tight tolerance.
- ``kl``/``objective``: the Kullback-Leibler divergence of Definition
  "Kullback-Leibler divergence" and the entropic objective eps*KL(pi|K).
- ``monotone_w2sq``: the closed-form 1D optimal transport cost (monotone
  rearrangement, north-west corner rule on sorted points).
"""
import numpy as np
from scipy.special import logsumexp


def kl(p, q):
    """KL(p|q) = sum phi(p/q) q with phi(s) = s log s - s + 1; requires q > 0 where p > 0."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    pos = p > 0
    if np.any(q[pos] <= 0):
        return np.inf
    out = np.sum(q) - np.sum(p)
    out += np.sum(p[pos] * np.log(p[pos] / q[pos]))
    return float(out)


def kernel(C, mu, nu, eps):
    """K = exp(-c/eps) (mu x nu), the reference measure of the entropic problem."""
    return np.exp(-C / eps) * np.outer(mu, nu)


def objective(plan, C, mu, nu, eps):
    """eps * KL(plan | K)."""
    return eps * kl(plan, kernel(C, mu, nu, eps))


def sinkhorn(C, mu, nu, eps, tol=1e-13, max_iter=200000, f=None):
    """Log-domain Sinkhorn between mu and nu for the cost matrix C (absolute units).

    Plan pi = exp((f(x)+g(y)-C(x,y))/eps) mu(x) nu(y).  Starts from f (zero by
    default) with a Y-iteration; after each Y-iteration the L1 error of the
    X-marginal is compared with tol*|mu| and the solver stops there (so the
    Y-marginal holds).  Returns (f, g, plan, loops, err).
    """
    C = np.asarray(C, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    lmu = np.where(mu > 0, np.log(np.where(mu > 0, mu, 1.0)), -np.inf)
    lnu = np.where(nu > 0, np.log(np.where(nu > 0, nu, 1.0)), -np.inf)
    F = np.zeros(len(mu)) if f is None else np.asarray(f, dtype=np.float64) / eps
    Cs = C / eps
    err = np.inf
    for it in range(1, max_iter + 1):
        G = -logsumexp(F[:, None] - Cs + lmu[:, None], axis=0)
        Fh = -logsumexp(G[None, :] - Cs + lnu[None, :], axis=1)
        err = float(np.sum(mu * np.abs(np.exp(F - Fh) - 1.0)))
        if err <= tol * mu.sum() or it == max_iter:
            break
        F = np.where(mu > 0, Fh, F)
    plan = np.exp(F[:, None] + G[None, :] - Cs) * np.outer(mu, nu)
    return eps * F, eps * G, plan, it, err


def entropic_ot(C, mu, nu, eps, tol=1e-13, max_iter=200000):
    """Unique minimiser of eps*KL(pi|K) over Pi(mu, nu): Newton on the dual,
    falling back to Sinkhorn if Newton does not reach the tolerance."""
    try:
        with np.errstate(over="ignore", under="ignore", invalid="ignore"):
            P = entropic_ot_newton(C, mu, nu, eps)[2]
        if np.all(np.isfinite(P)) and (np.abs(P.sum(1) - mu).sum() + np.abs(P.sum(0) - nu).sum()
                                       <= 10 * tol * np.sum(mu)):
            return P
    except np.linalg.LinAlgError:
        pass
    return sinkhorn(C, mu, nu, eps, tol=tol, max_iter=max_iter)[2]


def dd_dense(C, mu, nu, eps, cells_a, cells_b, basic, pi0, n_half, tol=1e-13,
             max_iter=100000):
    """Algorithm 1 (entropic domain decomposition) on a dense plan.

    basic: list of index arrays (the basic cells X_i); cells_a / cells_b:
    lists of lists of basic-cell ids (the composite partitions).  Iteration l
    (1-based) uses A for odd l, B for even l.  On each composite cell J the
    Y-marginal nu_J of the previous plan restricted to X_J x Y is computed and
    the plan on X_J x Y is replaced by the entropic optimum between mu_J and
    nu_J.  Returns the list of plans [pi0, pi1, ..., pi_n].
    """
    C = np.asarray(C, dtype=np.float64)
    plans = [np.array(pi0, dtype=np.float64)]
    pi = plans[0]
    for ell in range(1, n_half + 1):
        cells = cells_a if ell % 2 == 1 else cells_b
        new = np.zeros_like(pi)
        for J in cells:
            xs = np.concatenate([basic[i] for i in J])
            nuJ = pi[xs, :].sum(axis=0)
            sup = np.nonzero(nuJ > 0)[0]
            p = entropic_ot(C[np.ix_(xs, sup)], mu[xs], nuJ[sup], eps, tol=tol,
                            max_iter=max_iter)
            new[np.ix_(xs, sup)] = p
        pi = new
        plans.append(pi)
    return plans


def grid_cost(H, W, h, p=2.0):
    """Dense |x-y|^p between the pixel centres of an H x W grid with spacing h."""
    r, c = np.divmod(np.arange(H * W), W)
    d2 = ((r[:, None] - r[None, :]) ** 2 + (c[:, None] - c[None, :]) ** 2).astype(np.float64)
    if p == 2.0:
        return d2 * h * h
    return np.sqrt(d2) ** p * h ** p


def grid_partitions(H, W, s):
    """Basic s x s cells and the composite partitions A (2x2 blocks) and B
    (2x2 blocks offset by one basic cell), in the same ordering as the oracle."""
    bh, bw = H // s, W // s
    basic = []
    for b in range(bh * bw):
        br, bc = divmod(b, bw)
        rr, cc = np.meshgrid(np.arange(br * s, br * s + s), np.arange(bc * s, bc * s + s),
                             indexing="ij")
        basic.append((rr * W + cc).ravel())

    def groups(n, part):
        if part == 0:
            return [[2 * g, 2 * g + 1] for g in range(n // 2)]
        out = []
        for g in range(n // 2 + 1):
            out.append([r for r in (2 * g - 1, 2 * g) if 0 <= r < n])
        return out

    parts = []
    for part in (0, 1):
        cells = []
        for rg in groups(bh, part):
            for cg in groups(bw, part):
                cells.append([r * bw + c for r in rg for c in cg])
        parts.append(cells)
    return basic, parts[0], parts[1]


def monotone_w2sq(x, a, y, b, p=2.0):
    """W2^2 between sum a_i delta_{x_i} and sum b_j delta_{y_j} on the line
    (north-west corner rule on the sorted supports: the optimal plan of a
    strictly convex cost h(x-y) is the monotone one); with p != 2 the cost
    of that plan for |x-y|^p."""
    ix, iy = np.argsort(x), np.argsort(y)
    x, a = np.asarray(x, float)[ix], np.asarray(a, float)[ix]
    y, b = np.asarray(y, float)[iy], np.asarray(b, float)[iy]
    i = j = 0
    ra, rb = a[0], b[0]
    tot = 0.0
    while i < len(x) and j < len(y):
        m = min(ra, rb)
        tot += m * abs(x[i] - y[j]) ** p
        ra -= m
        rb -= m
        if ra <= 1e-300:
            i += 1
            if i < len(x):
                ra = a[i]
        if rb <= 1e-300:
            j += 1
            if j < len(y):
                rb = b[j]
    return tot


def entropic_ot_newton(C, mu, nu, eps, tol=1e-15, max_iter=200, warm=50):
    """Entropic optimum by damped Newton on the concave dual
        D(F,G) = <mu,F> + <nu,G> - sum exp(F(x)+G(y)-C(x,y)/eps) mu(x) nu(y)
    (Definition "Dual problem" in the variables F = log u, G = log v), with
    the gauge G[0] = 0 and a tiny Levenberg-Marquardt shift for nearly
    singular Hessians.  Started from a few log-domain Sinkhorn iterations;
    independent of the Sinkhorn stopping rule and quadratically convergent,
    so it is used for exact solves of small problems.  Returns (f, g, plan)."""
    C = np.asarray(C, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    nx, ny = C.shape
    Cs = C / eps
    lmn = np.log(mu)[:, None] + np.log(nu)[None, :]
    F = np.zeros(nx)
    G = np.zeros(ny)
    for _ in range(warm):
        G = -logsumexp(F[:, None] - Cs + np.log(mu)[:, None], axis=0)
        F = -logsumexp(G[None, :] - Cs + np.log(nu)[None, :], axis=1)
    F += G[0]
    G -= G[0]

    def plan(F, G):
        return np.exp(F[:, None] + G[None, :] - Cs + lmn)

    def dual(F, G):
        return mu @ F + nu @ G - np.sum(plan(F, G))

    for _ in range(max_iter):
        P = plan(F, G)
        gx, gy = mu - P.sum(1), nu - P.sum(0)
        if np.abs(gx).sum() + np.abs(gy).sum() <= tol * mu.sum():
            break
        Hm = np.zeros((nx + ny - 1, nx + ny - 1))
        Hm[:nx, :nx] = np.diag(P.sum(1))
        Hm[nx:, nx:] = np.diag(P.sum(0)[1:])
        Hm[:nx, nx:] = P[:, 1:]
        Hm[nx:, :nx] = P[:, 1:].T
        grad = np.concatenate([gx, gy[1:]])
        Hm += np.eye(len(grad)) * (1e-13 * np.abs(np.diag(Hm)).max() + 1e-300)
        step = np.linalg.solve(Hm, grad)
        d0 = dual(F, G)
        t = 1.0
        ok = False
        while t > 1e-10:
            F2 = F + t * step[:nx]
            G2 = G.copy()
            G2[1:] += t * step[nx:]
            d2 = dual(F2, G2)
            if np.isfinite(d2) and d2 >= d0 - 1e-15 * abs(d0):
                ok = True
                break
            t *= 0.5
        if not ok:
            break
        F, G = F2, G2
    return eps * F, eps * G, plan(F, G)
