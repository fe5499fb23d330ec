"""A hard composite cell of the uneven batch, on the CPU oracle.

The cell (tests/golden/hard_cell_config4.json, written by
tests/golden/make_hard_cell.py from the oracle alone) has its whole
Y-support nu_J 150-180 pixels away from its 8x8 block at eps = h^2/2.  Every
support point is then served by the one block pixel nearest to it, the
couplings between block pixels nearly vanish, and the cell Sinkhorn of
Remark "Sinkhorn algorithm" crawls (the oracle's default mode took tens of
thousands of loops; the Newton system is nearly singular).  Doubling eps
for the cell and returning to eps from that solution (the safeguard of
Sec. 7.4) solves it in a few hundred loops each, so the solvers treat a cell
that is not converged after `safeguard_after` loops (default 1024) as
failing.  Regression test: the early safeguard solves the cell to the same
stopping rule (Sec. 6.2), and to the same fixed point as a solve run far
below the tolerance."""
import json
import os

import numpy as np

from oracle import ddo

HERE = os.path.dirname(os.path.abspath(__file__))


def _cell():
    with open(os.path.join(HERE, "golden", "hard_cell_config4.json")) as f:
        d = json.load(f)
    a = {k: np.array(d[k]) for k in ("xr", "xc", "mu", "yr", "yc", "nu", "F0")}
    return d, a


def _solve(a, lam, tol, max_iter, F, accel=1, newton_after=384):
    return ddo.cell_solve(a["xr"], a["xc"], a["mu"], a["yr"], a["yc"], a["nu"], lam, tol,
                          max_iter, F0=F, accel=accel, newton_after=newton_after)


def _safeguarded(a, lam, tol, cap0=1024, cap=50000):
    r = _solve(a, lam, tol, cap0, a["F0"].copy())
    if r["rc"] == 0:
        return r, r["loops"], False
    r2 = _solve(a, 0.5 * lam, tol, cap, 0.5 * a["F0"])
    r3 = _solve(a, lam, tol, cap, 2.0 * r2["F"])
    return r3, r["loops"] + r2["loops"] + r3["loops"], True


def test_hard_cell_is_solved_by_the_early_safeguard():
    d, a = _cell()
    lam, tol = d["lam"], d["tol"]
    assert d["loops_default_mode"] > 10000
    # far support: no support point within 8 pixels of the block
    dr = np.maximum(0, np.maximum(a["xr"].min() - a["yr"], a["yr"] - a["xr"].max()))
    dc = np.maximum(0, np.maximum(a["xc"].min() - a["yc"], a["yc"] - a["xc"].max()))
    assert np.hypot(dr, dc).min() > 8
    r, loops, used = _safeguarded(a, lam, tol)
    print("hard cell: stored default-mode loops", d["loops_default_mode"], "early safeguard",
          loops, flush=True)
    assert used and r["rc"] == 0 and r["err"] <= tol
    assert loops <= 5000
    # exact Y-marginal of the returned plan (up to the rounding of exponents
    # of size lam |x-y|^2 ~ 6e4: relative 1e-9), X-marginal within the tolerance
    P = r["plan"]
    assert np.all(np.abs(P.sum(axis=0) - a["nu"]) <= 1e-9 * a["nu"] + 1e-30)
    assert np.abs(P.sum(axis=1) - a["mu"]).sum() <= tol
    # the same fixed point as a solve a hundred times below the tolerance
    # (the X-error cannot go much lower: the rounding of the exponents above
    # leaves ~1e-13 of |mu_J| = 9e-6)
    rt, _, _ = _safeguarded(a, lam, tol * 1e-2)
    assert rt["rc"] == 0
    cost = lambda Q: float(np.sum(Q * ((a["xr"][:, None] - a["yr"][None, :]) ** 2
                                       + (a["xc"][:, None] - a["yc"][None, :]) ** 2)))
    c, ct = cost(P), cost(rt["plan"])
    assert abs(c - ct) <= 1e-3 * ct
    assert np.abs(P - rt["plan"]).sum() <= 4 * tol
