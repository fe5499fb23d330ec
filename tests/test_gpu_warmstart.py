"""Learned warm start on the GPU: the cell features and training targets that
the library collects, recomputed on the CPU from the exported states; and a
small network trained on the GPU by the library's kernels, used as the warm
start of a fresh problem: same accuracy as the plain method (the network only
moves the starting point; the stopping test is unchanged), and the loop counts
of both runs are reported.
"""
import numpy as np
import pytest

from paper_2001_10986_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _cpu_rows(exp_prev, exp_after, mu_l, H, W, h, eps, cells_basic, part, cell_ids):
    """Features and targets (as defined in include/dd_mlp.h) of the given cells."""
    lam = h * h / eps
    bw = W // 4
    rp, col, val = exp_prev["row_ptr"], exp_prev["col"], exp_prev["val"]
    Ap, Aa = exp_prev["alpha_a" if part == 0 else "alpha_b"].ravel(), \
        exp_after["alpha_a" if part == 0 else "alpha_b"].ravel()
    X, T, M = [], [], []
    for cid in cell_ids:
        bs = [b for b in cells_basic[cid] if b >= 0]
        brs = [b // bw for b in bs]
        bcs = [b % bw for b in bs]
        R0 = 4 * (2 * ((max(brs) + part) // 2) - part)
        C0 = 4 * (2 * ((max(bcs) + part) // 2) - part)
        present = set(bs)
        mu_blk = np.zeros(64)
        act = np.zeros(64, bool)
        for i in range(8):
            for j in range(8):
                b = ((R0 + i) // 4) * bw + (C0 + j) // 4 if 0 <= R0 + i < H and 0 <= C0 + j < W else -1
                if b in present:
                    mu_blk[8 * i + j] = mu_l[R0 + i, C0 + j]
        ys = {}
        for b in bs:
            for q in range(rp[b], rp[b + 1]):
                ys[col[q]] = ys.get(col[q], 0.0) + val[q]
        keys = np.array(sorted(ys))
        nuJ = np.array([ys[k] for k in keys])
        yr, yc = np.divmod(keys, W)
        mm, nm = mu_blk.sum(), nuJ.sum()
        ii, jj = np.divmod(np.arange(64), 8)
        dr = int(np.rint((nuJ * (yr - R0)).sum() / nm - (mu_blk * ii).sum() / mm))
        dc = int(np.rint((nuJ * (yc - C0)).sum() / nm - (mu_blk * jj).sum() / mm))
        f = np.zeros(768)
        f[:64] = 64 * mu_blk / mm
        wr, wc = yr - (R0 - 8 + dr), yc - (C0 - 8 + dc)
        inside = (wr >= 0) & (wr < 24) & (wc >= 0) & (wc < 24)
        f[64 + wr[inside] * 24 + wc[inside]] = 256 * nuJ[inside] / nm
        f[640] = np.log(lam)
        f[641] = nuJ[~inside].sum() / nm
        f[642], f[643] = dr / 8, dc / 8
        act = mu_blk > 0
        px = (R0 + ii) * W + (C0 + jj)
        ramp = 2 * lam * ((ii - 3.5) * dr + (jj - 3.5) * dc)

        def centred(alpha):
            F = np.where(act, alpha[np.where(act, px, 0)] / eps + ramp, 0.0)
            return np.where(act, F - F[act].mean(), 0.0)
        f0, f1 = centred(Ap), centred(Aa)
        f[644:708] = f0 / (16 * lam)
        X.append(f)
        T.append((f1 - f0) / (16 * lam))
        M.append(act.astype(float))
    return np.array(X), np.array(T), np.array(M)


def test_collected_samples_match_cpu_recompute(torch):
    from oracle import ddo
    from paper_2001_10986_amd import dd
    N = 64
    mu, nu = datagen.small_pair(N, 4, seed=9)
    eps = 1.0 / N ** 2
    g = dd.Problem(mu, nu, [(0, eps, 4)], s=4, n_levels=1)
    o = ddo.Oracle(mu, nu, s=4, n_levels=1, eps=eps)
    for k in range(6):  # from the product coupling every union is the whole image
        g.half_iterate(k & 1)
    for part in (0, 1, 0):
        prev = g.export()
        g.half_iterate(part)
        after = g.export()
        cap = 4096
        X = torch.zeros((cap, 768), device="cuda")
        T = torch.zeros((cap, 64), device="cuda")
        M = torch.zeros((cap, 64), device="cuda")
        ids = torch.zeros(cap, dtype=torch.int32, device="cuda")
        n = g.collect_cells(X, T, M, ids)
        r = g.cell_results()
        # every converged cell whose union has at most 8192 points, once
        rp, col = prev["row_ptr"], prev["col"]
        cb = o.cells(part)

        def union_size(k):
            bs = [b for b in cb[k] if b >= 0]
            return len(set(np.concatenate([col[rp[b]:rp[b + 1]] for b in bs]).tolist()))
        exp_cells = {k for k in range(len(r["status"]))
                     if r["status"][k] == 0 and union_size(k) <= 8192}
        idn = ids[:n].cpu().numpy()
        assert n > 0 and len(idn) == len(set(idn.tolist())) and set(idn.tolist()) == exp_cells
        Xc, Tc, Mc = _cpu_rows(prev, after, mu, N, N, 1.0 / N, eps, o.cells(part), part, idn)
        Xg, Tg, Mg = (a[:n].cpu().numpy().astype(np.float64) for a in (X, T, M))
        assert np.abs(Xg - Xc).max() < 1e-5 * max(1.0, np.abs(Xc).max())
        assert (Mg == Mc).all()
        assert np.abs(Tg - Tc).max() < 1e-4 * max(1.0, np.abs(Tc).max())


def test_learned_warm_start_keeps_accuracy(torch):
    from paper_2001_10986_amd import dd, mlp, warmstart
    X, T, M = warmstart.generate(4, 200_000)
    assert X.shape[0] > 10_000
    net = mlp.MLP(warmstart.N_IN, warmstart.N_OUT, warmstart.WIDTH, seed=2)
    before = warmstart.mean_loss(net, X, T, M)
    warmstart.train(net, X, T, M, 400, batch=2048)
    after = warmstart.mean_loss(net, X, T, M)
    assert after < 0.2 * before
    # a fresh pair (evaluation seeds) on two levels
    mu = datagen.blob_image(128, 128, 8, 7000)
    nu = datagen.blob_image(128, 128, 8, 7001)
    sched = datagen.eps_schedule(128, 2)
    res = {}
    for name, (pol, thr) in {"plain": (0, 0.0), "learned": (warmstart.POLICY, warmstart.MIN_RMS),
                             "every_sweep": (2, 0.0)}.items():
        g = dd.Problem(torch.from_numpy(mu).cuda(), torch.from_numpy(nu).cuda(), sched, s=4,
                       n_levels=2)
        if pol:
            g.set_warm_start(net, pol, thr)
        rs = g.run_schedule()
        res[name] = (rs, g.cost(), g.warm_start_count())
        g.close()
    p = res["plain"][1]
    for name, (rs, c, wc) in res.items():
        print(name, "loops", rs["loops_total"], "newton", rs["n_newton"], "warm", wc,
              "cost", c["cost"], "err_x", c["err_x"], flush=True)
        assert rs["n_failed"] == 0 and c["err_x"] <= 1e-5 and c["err_y"] <= 1e-5
        assert abs(c["cost"] - p["cost"]) <= 1e-5 * p["cost"]
    assert res["learned"][2][0] > 0 and res["every_sweep"][2][1] > 0


def test_prediction_of_the_converged_change_restarts_at_the_solution(torch):
    # Pins the apply step of the learned start: the targets collected from a
    # sweep (the change of the centred potential that each solve made) are
    # handed back as the prediction for the same sweep from the same state.
    # Every such cell then starts at its converged potential up to a
    # constant, so its solve stops after the first loop with the same plan
    # and potential; a wrong sign, scale, centring or cell index would send
    # it away from the solution.
    from paper_2001_10986_amd import dd
    N = 64
    mu, nu = datagen.small_pair(N, 4, seed=29)
    # two levels down to eps = 2 h^2 (unions <= 8192 points), then the
    # change to eps = h^2: the next sweep's cells are away from their solution
    sched = datagen.eps_schedule(N, 2)
    eps = sched[-1][1]
    g = dd.Problem(mu, nu, sched[:-1], s=4, n_levels=2)
    g.run_schedule()
    g.set_eps(eps)
    part = 0
    s0 = g.export()
    g.half_iterate(part)
    r1 = g.cell_results()
    e1 = g.export()
    nc = len(r1["loops"])
    X = torch.zeros((nc, 768), device="cuda")
    T = torch.zeros((nc, 64), device="cuda")
    M = torch.zeros((nc, 64), device="cuda")
    ids = torch.zeros(nc, dtype=torch.int32, device="cuda")
    n = g.collect_cells(X, T, M, ids)
    assert n >= 20
    g.import_state(s0["level"], s0["eps"], s0["row_ptr"], s0["col"], s0["val"], s0["alpha_a"],
                   s0["alpha_b"])
    Y = torch.zeros((nc, 64), device="cuda")
    Y[ids[:n].long()] = T[:n]
    g.set_warm_prediction(Y, 0.0)
    g.half_iterate(part)
    r2 = g.cell_results()
    e2 = g.export()
    warm = ids[:n].cpu().numpy()
    print("cells", nc, "given a prediction", n, "loops first run", int(r1["loops"][warm].sum()),
          "restart", int(r2["loops"][warm].sum()), "max", int(r2["loops"][warm].max()), flush=True)
    assert r1["loops"][warm].min() >= 2
    assert r2["loops"][warm].max() <= 2
    # the other cells started where they did the first time
    rest = np.setdiff1d(np.arange(nc), warm)
    assert np.array_equal(r1["loops"][rest], r2["loops"][rest])
    # potentials: the converged ones up to one constant per cell (cell
    # geometry from the oracle's partition tables)
    from oracle import ddo
    cells_p = ddo.Oracle(mu, nu, s=4, n_levels=1, eps=eps).cells(part)  # 64x64 geometry
    d = (e2["alpha_a"] - e1["alpha_a"]) / eps
    bw = N // 4
    for k in warm:
        blk = np.concatenate([d[4 * (b // bw):4 * (b // bw) + 4, 4 * (b % bw):4 * (b % bw) + 4].ravel()
                              for b in cells_p[k] if b >= 0])
        assert np.ptp(blk) < 1e-5, (k, np.ptp(blk))
    # and the plans: the basic marginals of both runs
    bm1 = np.zeros((len(e1["row_ptr"]) - 1, N * N))
    bm2 = np.zeros_like(bm1)
    for bm, e in ((bm1, e1), (bm2, e2)):
        for b in range(bm.shape[0]):
            bm[b, e["col"][e["row_ptr"][b]:e["row_ptr"][b + 1]]] = \
                e["val"][e["row_ptr"][b]:e["row_ptr"][b + 1]]
    assert np.abs(bm1 - bm2).max() < 1e-5 * bm1.sum(axis=1).max()
