"""The C-ABI library loads and exports every function declared in include/*.h, and the
host-side recipes (schedules, generators, bench traffic guard) hold (CPU only)."""
import ctypes
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in ("dd.h", "dd_mlp.h", "dd_single.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(dd_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("dd_init", "dd_half_iterate", "dd_set_eps", "dd_refine", "dd_run_schedule",
              "dd_cost", "dd_export_plan", "dd_import_state", "dd_free", "dd_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2001_10986_amd import dd
    lib = ctypes.CDLL(dd.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(dd.EXPORTED) <= set(_declared())


def test_single_options_default_without_gpu():
    from paper_2001_10986_amd import dd
    o = dd.SingleOptions()
    dd.lib.dd_single_options_default(ctypes.byref(o))
    assert o.err_tol == 1e-7 and o.theta == 1e-10 and o.err_norm == dd.DD_SINGLE_LINF
    assert o.cost_p == 2.0 and o.check_every == 16


def test_options_default_without_gpu():
    from paper_2001_10986_amd import dd
    o = dd.Options()
    dd.lib.dd_options_default(ctypes.byref(o))
    assert o.err_tol == 1e-5 and o.trunc_threshold == 1e-15 and o.max_sinkhorn_iter == 50000
    assert o.safeguard == 1 and o.inputs_on_device == 0 and o.accel == 1 and o.newton_after == 384
    assert o.precision == dd.DD_PREC_SPLIT and o.cost_p == 2.0 and o.safeguard_after == 1024


def test_probe_peaks_rejects_null_without_gpu():
    # the argument check comes before any device call
    from paper_2001_10986_amd import dd
    assert dd.lib.dd_probe_peaks(None) == -1  # DD_EINVAL
    assert dd.lib.dd_probe_last_error() == b"null output"


def test_schedule_recipe():
    from paper_2001_10986_amd import datagen
    st = datagen.eps_schedule(256, 3)
    # levels 64 -> 128 -> 256, eps 1 -> (1/256)^2, 4 half-iterations on every first stage
    assert st[0] == (0, 1.0, 4) and st[-1] == (2, 2.0 ** -16, 4)
    assert [s for s in st if s[0] == 1] == [(1, 2.0 ** -13, 4), (1, 2.0 ** -14, 2),
                                            (1, 2.0 ** -15, 2)]
    assert sum(s[2] for s in datagen.eps_schedule(1024, 5)) == 62


def test_generator_is_deterministic():
    from paper_2001_10986_amd import datagen
    a = datagen.blob_image(32, 32, 4, 1000)
    b = datagen.blob_image(32, 32, 4, 1000)
    assert a.dtype.name == "float64" and abs(a.sum() - 1) < 1e-14
    assert (a == b).all() and (a > 0).all()
    assert not (a == datagen.blob_image(32, 32, 4, 1001)).all()


def test_uneven_batch_recipe():
    from paper_2001_10986_amd import datagen
    pairs = datagen.config4_pairs(8)
    assert len(pairs) == 8
    for mu, nu, cfg in pairs:
        N = mu.shape[0]
        assert mu.shape == nu.shape == (N, N) and N in (64, 128, 256, 512)
        assert abs(mu.sum() - 1) < 1e-12 and abs(nu.sum() - 1) < 1e-12
        # coarsest level 64 px, finest eps (1/N)^2
        assert cfg["n_levels"] == int(np.log2(N // 64)) + 1
        assert N >> (cfg["n_levels"] - 1) == 64
        assert cfg["stages"][-1][0] == cfg["n_levels"] - 1
        assert abs(cfg["stages"][-1][1] - 1.0 / N ** 2) < 1e-15
    # the same recipe every time
    again = datagen.config4_pairs(8)
    assert all((a[0] == b[0]).all() for a, b in zip(pairs, again))


def test_bench_traffic_only_for_the_profiled_kernel_build(tmp_path):
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "bench", os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                              "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    # other workloads and unprofiled kernels report no traffic
    assert bench.kernel_traffic("solve_reg_16w", False) is None
    assert bench.kernel_traffic("union", True) is None
    # a source that does not match the profiled hash reports none either
    bench.ROOT = str(tmp_path)
    src = tmp_path / "paper_2001_10986_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "dd_kernels.hip").write_text("// changed\n")
    assert bench.kernel_traffic("solve_reg_16w", True) is None
