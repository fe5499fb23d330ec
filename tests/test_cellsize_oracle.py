"""Basic-cell size study on the FP64 oracle (CPU): Sec. 7.1 "Basic and
composite partitions" says that small cells make the composite problems
easy but need more cells and more iterations, large cells the reverse.  On
the paper's protocol (here from 16x16 layers, so that s = 8 fits) with the
same number of iterations, the relative PD gap falls as s grows while the
number of cell solves falls too; s = 8 is not run on the GPU (its 16x16
composite cells do not fit the solvers' 8x8 block)."""
import numpy as np

from oracle import certificate as cert
from oracle import dense, ddo
from paper_2001_10986_amd import datagen


def test_gap_and_solves_against_cell_size():
    N = 64
    mu, nu = datagen.small_pair(N, 8, seed=11)
    stages, nlev = datagen.paper_schedule(N, coarsest=16)
    C = dense.grid_cost(N, N, 1.0 / N)
    res = {}
    for s in (2, 4, 8):
        o = ddo.Oracle(mu, nu, s=s, n_levels=nlev, eps=stages[0][1], err_tol=1e-4)
        st = o.run_schedule(stages)
        e = o.export()
        basic, ca, cb = dense.grid_partitions(N, N, s)
        r = cert.certificate(e["alpha_a"], e["alpha_b"], o.cost()["obj"], C, mu.ravel(),
                             nu.ravel(), stages[-1][1], basic, ca, cb)
        res[s] = (r["rel_gap"], st["n_cells"], st["loops_total"], o.cost()["cost"])
        print(s, res[s], flush=True)
    assert res[2][0] > res[4][0] > res[8][0] > 0
    assert res[2][1] > res[4][1] > res[8][1]
    # s = 4 and s = 8 end at nearly the same plan; s = 2 has not converged
    assert abs(res[4][3] - res[8][3]) < 1e-4 * res[8][3] < abs(res[2][3] - res[8][3])
