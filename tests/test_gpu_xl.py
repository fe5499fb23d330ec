"""The paper's largest instance on the GPU, through the C-ABI.

A 2048x2048 blob pair (the largest image size of the paper's summary table of
the quantitative evaluation) on six levels 64 -> 2048, with the eps schedule
carried on to a quarter of the squared finest pixel spacing (the paper's two
extra iterations at eps = 0.25 in pixel units, Sec. 7.1).  At this eps the
kernel entries span a wider range than at (1/N)^2, which exercises the FP32
exponent range of the absorbed tiles.  Checked: properties that hold at any
size on the whole result, then one more finest-level sweep of partition A
compared cell by cell with the FP64 oracle, from the same state, on a random
sample of cells.
"""
import os
import time

import numpy as np
import pytest

from paper_2001_10986_amd import datagen

pytestmark = pytest.mark.gpu


def _check_rows(e, H, W, nb):
    rp, col, val = e["row_ptr"], e["col"], e["val"]
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and len(col) == rp[-1]
    assert col.min() >= 0 and col.max() < H * W
    assert np.all(np.isfinite(val)) and val.min() > 0
    # strictly increasing columns inside every basic-cell row
    inc = np.diff(col) > 0
    first = np.zeros(len(col), dtype=bool)
    first[rp[:-1][np.diff(rp) > 0]] = True
    assert np.all(inc | first[1:])
    assert len(rp) == nb + 1


def test_2048_quarter_eps_schedule_and_sampled_cells(capsys):
    from oracle import ddo
    from paper_2001_10986_amd import dd
    mu, nu, cfg = datagen.config3_pair(N=2048, final_factor=0.25)
    H, W = mu.shape
    s = cfg["s"]
    assert cfg["n_levels"] == 6 and cfg["stages"][-1][1] == 0.25 / 2048 ** 2
    n_half = sum(st[2] for st in cfg["stages"])
    print(f"2048x2048, {len(cfg['stages'])} stages, {n_half} half-iterations", flush=True)
    g = dd.Problem(mu, nu, cfg["stages"], s=s, n_levels=cfg["n_levels"])
    t = time.perf_counter()
    rs = g.run_schedule()
    c = g.cost()
    dt = time.perf_counter() - t
    print(f"schedule {dt:.2f} s, cell solves {rs['n_cell_solves']}, W2^2 {c['cost']:.10g}, "
          f"err_x {c['err_x']:.3g}, err_y {c['err_y']:.3g}, failed {rs['n_failed']}",
          flush=True)
    assert rs["n_half_iters"] == n_half and rs["n_failed"] == 0
    assert c["err_x"] <= 1e-5 and c["err_y"] <= 1e-5
    e = g.export()
    info = g.level_info()
    nb = info["n_basic"]
    assert info["H"] == H and info["W"] == W and nb == (H // s) * (W // s)
    _check_rows(e, H, W, nb)
    rows = np.repeat(np.arange(nb), np.diff(e["row_ptr"]))
    rm = np.bincount(rows, weights=e["val"], minlength=nb)
    blk = mu.reshape(H // s, s, W // s, s).sum(axis=(1, 3)).ravel()
    assert np.abs(rm - blk).sum() <= 2 * c["mass_drift"] + 1e-12
    colm = np.bincount(e["col"], weights=e["val"], minlength=H * W)
    assert np.abs(colm - nu.ravel()).sum() <= 1e-5
    pd = g.certificate()
    print(f"relative PD gap {pd['rel_gap']:.4e}", flush=True)
    # weak duality up to the marginal tolerance (3.0e-3 measured on this
    # schedule, whose hierarchy starts at 64x64; the bar against the paper's
    # table is tested with its own protocol in test_gpu_certificate.py)
    assert pd["n_uncovered"] == 0 and 0 < pd["rel_gap"] and pd["status"] == 0
    o = ddo.Oracle(mu, nu, s=s, n_levels=cfg["n_levels"], eps=cfg["stages"][0][1],
                   n_threads=min(16, os.cpu_count() or 1))
    o.import_state(e["level"], e["eps"], e["row_ptr"], e["col"], e["val"], e["alpha_a"],
                   e["alpha_b"])
    del e, rows, colm
    n_cells = o.level_info()["n_cells_a"]
    assert n_cells == (H // (2 * s)) * (W // (2 * s))
    mask = np.zeros(n_cells, dtype=np.uint8)
    mask[np.random.default_rng(2).permutation(n_cells)[:768]] = 1
    o.half_iterate(0, mask)
    sg = g.half_iterate(0)
    assert sg["n_failed"] == 0
    rg, ro = g.cell_results(), o.cell_results(0)
    m = mask.astype(bool)
    rel = np.abs(rg["cost"][m] - ro["cost"][m]) / np.maximum(np.abs(ro["cost"][m]), 1e-300)
    lg, lo = int(rg["loops"][m].sum()), int(ro["loops"][m].sum())
    print(f"sampled cells {int(m.sum())}: max rel cost diff {rel.max():.3g}, loops gpu {lg} "
          f"oracle {lo}", flush=True)
    assert np.all(np.abs(rg["cost"][m] - ro["cost"][m]) <= 2e-5 * np.abs(ro["cost"][m]) + 1e-18)
    assert abs(lg - lo) <= 0.02 * lo + 16
    o.close()
    g.close()
