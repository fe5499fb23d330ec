"""Batched sweeps (dd_batch_*) through the C-ABI on the GPU.

A batch runs the cells of several problems through the same launches; every
cell is still solved by one workgroup with the same code and the same
reduction order, so each problem's state after a batched sweep must equal,
bit for bit, the state its own dd_half_iterate gives.  The single-problem
path itself is checked against the FP64 oracle in test_gpu_parity.py; one
case here compares a batched problem with the oracle directly.
"""
import numpy as np
import pytest

from paper_2001_10986_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    from paper_2001_10986_amd import dd as m
    return m


def _states_equal(a, b):
    ea, eb = a.export(), b.export()
    assert ea["level"] == eb["level"] and ea["eps"] == eb["eps"]
    for k in ("row_ptr", "col", "val", "alpha_a", "alpha_b"):
        assert np.array_equal(ea[k], eb[k]), k


def _mixed_problems(dd, cases):
    return [dd.Problem(mu, nu, st, s=4, n_levels=nl) for mu, nu, st, nl in cases]


def _cases():
    out = []
    for N, seed in ((16, 31), (32, 33), (64, 35), (32, 37)):
        mu, nu = datagen.small_pair(N, 3, seed=seed)
        out.append((mu, nu, [(0, 4.0 / N ** 2, 6)], 1))
    return out


def test_batched_sweeps_equal_single_sweeps(dd):
    cases = _cases()
    single = _mixed_problems(dd, cases)
    batched = _mixed_problems(dd, cases)
    b = dd.Batch(batched)
    for ell in range(4):
        sb = b.half_iterate(ell % 2)
        for i, g in enumerate(single):
            ss = g.half_iterate(ell % 2)
            for k in ("n_cells", "loops_total", "loops_max", "n_newton", "nnz", "entry_evals"):
                assert sb[i][k] == ss[k], (i, k)
            assert sb[i]["cost"] == ss["cost"]
    for g, h in zip(single, batched):
        _states_equal(g, h)
    assert b.info()["n_sweeps"] == 4
    b.close()


def test_batch_graph_replays_equal_eager(dd):
    cases = _cases()
    eager = _mixed_problems(dd, cases)
    graphed = _mixed_problems(dd, cases)
    be, bg = dd.Batch(eager), dd.Batch(graphed, graph=True)
    for ell in range(6):
        se = be.half_iterate(ell % 2)
        sg = bg.half_iterate(ell % 2)
        for i in range(len(cases)):
            assert se[i]["loops_total"] == sg[i]["loops_total"]
            assert se[i]["cost"] == sg[i]["cost"]
        for g, h in zip(eager, graphed):
            _states_equal(g, h)
    info = bg.info()
    # the shape stays fixed after the first sweep of each partition (buffer
    # sizes may grow once with the support), so most sweeps are replays
    assert info["n_sweeps"] == 6 and 1 <= info["n_captures"] <= 4
    be.close()
    bg.close()


def test_batch_schedule_uneven_equals_single(dd):
    # problems with different sizes, level counts and schedule lengths; the
    # batch runs them in lockstep and drops finished ones
    specs = [(32, 1, 41), (64, 2, 43), (128, 2, 45), (64, 1, 47)]
    cases = []
    for N, nl, seed in specs:
        mu, nu = datagen.small_pair(N, 4, seed=seed)
        st = datagen.eps_schedule(N, nl, eps_start=1.0 / 16)
        cases.append((mu, nu, st, nl))
    single = _mixed_problems(dd, cases)
    rs_single = [g.run_schedule() for g in single]
    for graph in (False, True):
        batched = _mixed_problems(dd, cases)
        b = dd.Batch(batched, graph=graph)
        rs = b.run_schedule()
        for i, g in enumerate(single):
            assert rs[i]["n_half_iters"] == rs_single[i]["n_half_iters"]
            assert rs[i]["loops_total"] == rs_single[i]["loops_total"]
            assert rs[i]["n_cell_solves"] == rs_single[i]["n_cell_solves"]
            _states_equal(g, batched[i])
            c = batched[i].cost()
            assert c["err_x"] <= 1e-5 and c["err_y"] <= 1e-5
        n_sweeps = b.info()["n_sweeps"]
        assert n_sweeps == max(r["n_half_iters"] for r in rs_single)
        b.close()


def test_batched_problem_matches_oracle(dd):
    from oracle import ddo
    N = 32
    mu, nu = datagen.small_pair(N, 3, seed=51)
    eps = 4.0 / N ** 2
    other = datagen.small_pair(64, 3, seed=53)
    g = dd.Problem(mu, nu, [(0, eps, 4)], s=4, n_levels=1)
    h = dd.Problem(other[0], other[1], [(0, 4.0 / 64 ** 2, 4)], s=4, n_levels=1)
    o = ddo.Oracle(mu, nu, s=4, n_levels=1, eps=eps)
    b = dd.Batch([h, g])
    for ell in range(4):
        b.half_iterate(ell % 2)
        o.half_iterate(ell % 2)
    b.close()
    cg, co = g.cost(), o.cost()
    assert abs(cg["cost"] - co["cost"]) <= 1e-5 * abs(co["cost"])
    e, eo = g.export(), o.export()
    mg = np.zeros(N * N)
    mo = np.zeros(N * N)
    np.add.at(mg, e["col"], e["val"])
    np.add.at(mo, eo["col"], eo["val"])
    assert np.abs(mg - mo).sum() <= 1e-5


def test_batch_rules(dd):
    mu, nu = datagen.small_pair(16, 3, seed=61)
    g = dd.Problem(mu, nu, [(0, 4.0 / 256, 2)], s=4, n_levels=1)
    h = dd.Problem(mu, nu, [(0, 4.0 / 256, 2)], s=4, n_levels=1)
    with pytest.raises(dd.DDError):
        dd.Batch([g, g])
    b = dd.Batch([g, h])
    with pytest.raises(dd.DDError):
        g.half_iterate(0)  # the context belongs to the batch
    with pytest.raises(dd.DDError):
        dd.Batch([h])  # already in a batch
    b.half_iterate(0)
    b.close()
    g.half_iterate(1)  # back to its own sweeps


def test_autotune_leaves_state_and_results_unchanged(dd):
    # the number of workgroups per launch changes the speed only: after the
    # tuner (which runs the next sweep 12 times from a snapshot) the state is
    # the one before, and the following sweeps match an untuned problem bit
    # for bit
    mu, nu = datagen.small_pair(64, 4, seed=71)
    st = [(0, 4.0 / 64 ** 2, 4)]
    g = dd.Problem(mu, nu, st, s=4, n_levels=1)
    h = dd.Problem(mu, nu, st, s=4, n_levels=1)
    g.half_iterate(0)
    h.half_iterate(0)
    before = g.export()
    best, tried = g.autotune(1, reps=1)
    after = g.export()
    for k in ("row_ptr", "col", "val", "alpha_a", "alpha_b"):
        assert np.array_equal(before[k], after[k]), k
    assert 10 <= len(tried) <= 16
    key = ("solver_per_cu", "newton_per_cu", "stream_wgs", "cells_per_wg")
    assert tuple(best[k] for k in key) in [tuple(t[k] for k in key) for t in tried]
    assert best["ms"] == min(t["ms"] for t in tried)
    for ell in (1, 0, 1):
        a, b = g.half_iterate(ell), h.half_iterate(ell)
        assert a["loops_total"] == b["loops_total"]
    _states_equal(g, h)
    with pytest.raises(dd.DDError):
        g.set_launch(0, 1)
    g.set_launch(8, 2, 64, 1)  # streamed-solver cap, one-shot workgroups: same results
    h.set_launch(8, 2, 0, 0)
    assert g.get_launch()["cells_per_wg"] == 1
    for ell in (0, 1):
        assert g.half_iterate(ell)["loops_total"] == h.half_iterate(ell)["loops_total"]
    _states_equal(g, h)


def test_batch_autotune_then_sweeps_equal_single(dd):
    cases = _cases()
    single = _mixed_problems(dd, cases)
    batched = _mixed_problems(dd, cases)
    b = dd.Batch(batched, graph=True)
    b.half_iterate(0)
    for g in single:
        g.half_iterate(0)
    best, tried = b.autotune(1, reps=1)
    assert 10 <= len(tried) <= 16
    for ell in (1, 0):
        b.half_iterate(ell)
        for g in single:
            g.half_iterate(ell)
    for g, h in zip(single, batched):
        _states_equal(g, h)
    b.close()


def test_batch_mixes_precisions(dd):
    # a split-precision and an FP64 problem in one batch: each keeps its own
    # solver path (the FP64 one's cells all go to the log-domain solver)
    mu, nu = datagen.small_pair(32, 3, seed=95)
    st = [(0, 4.0 / 32 ** 2, 4)]
    single = [dd.Problem(mu, nu, st, s=4, n_levels=1, precision=p)
              for p in (dd.DD_PREC_SPLIT, dd.DD_PREC_FP64)]
    batched = [dd.Problem(mu, nu, st, s=4, n_levels=1, precision=p)
               for p in (dd.DD_PREC_SPLIT, dd.DD_PREC_FP64)]
    b = dd.Batch(batched)
    for ell in range(4):
        sb = b.half_iterate(ell % 2)
        for i, g in enumerate(single):
            ss = g.half_iterate(ell % 2)
            assert sb[i]["cells_bin"] == ss["cells_bin"]
            assert sb[i]["loops_total"] == ss["loops_total"]
        assert sb[1]["cells_bin"][dd.N_BINS - 1] == sb[1]["n_cells"]
    for g, h in zip(single, batched):
        _states_equal(g, h)
    b.close()
