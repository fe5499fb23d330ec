"""ctypes binding of the HIP library (include/dd.h).

Argument marshalling only: every step of the method runs in the library's
kernels.  Importing this module loads ``libdd.so`` (built in-tree by
``paper_2001_10986_amd/csrc/build.py``) and raises if it is missing; there is
no CPU fallback.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdd.so")

DD_OK, DD_ENOTCONV = 0, 1
DD_EINVAL, DD_ENOMEM, DD_EHIP, DD_ECAPACITY, DD_ESTATE = -1, -2, -3, -4, -5

EXPORTED = ["dd_options_default", "dd_init", "dd_half_iterate", "dd_set_eps", "dd_refine",
            "dd_run_schedule", "dd_cost", "dd_export_plan", "dd_import_state",
            "dd_cell_results", "dd_level_info", "dd_free", "dd_last_error",
            "dd_mlp_create", "dd_mlp_free", "dd_mlp_last_error", "dd_mlp_shape",
            "dd_mlp_set_params", "dd_mlp_get_params", "dd_mlp_forward", "dd_mlp_forward_bf16",
            "dd_mlp_loss_grad", "dd_mlp_train_step", "dd_mlp_get_stream", "dd_set_warm_start",
            "dd_collect_cells", "dd_warm_start_count", "dd_batch_create",
            "dd_batch_half_iterate", "dd_batch_run_schedule", "dd_batch_schedule_step",
            "dd_batch_info", "dd_batch_free", "dd_set_launch", "dd_batch_set_launch",
            "dd_autotune", "dd_batch_autotune", "dd_get_launch",
            "dd_batch_last_error", "dd_certificate", "dd_cost_noalloc",
            "dd_set_warm_prediction", "dd_single_options_default", "dd_single_solve",
            "dd_single_last_error", "dd_probe_peaks", "dd_probe_last_error"]

DD_BATCH_GRAPH = 1
DD_PREC_SPLIT, DD_PREC_FP64 = 0, 1


class Stage(C.Structure):
    _fields_ = [("level", C.c_int), ("eps", C.c_double), ("n_half_iters", C.c_int)]


class Options(C.Structure):
    _fields_ = [("err_tol", C.c_double), ("trunc_threshold", C.c_double),
                ("max_sinkhorn_iter", C.c_int), ("safeguard", C.c_int), ("accel", C.c_int),
                ("newton_after", C.c_int), ("precision", C.c_int), ("inputs_on_device", C.c_int),
                ("timing", C.c_int), ("stream", C.c_void_p), ("cost_p", C.c_double),
                ("safeguard_after", C.c_int)]


N_KERNELS, N_BINS = 12, 7
KERNEL_NAMES = ["scan_cells", "union", "scan_out_bins", "solve_reg_1w", "solve_reg_2w",
                "solve_reg_4w", "solve_reg_8w", "solve_reg_16w", "solve_stream", "solve_big",
                "solve_newton", "stats"]


class IterStats(C.Structure):
    _fields_ = [("n_cells", C.c_int), ("loops_max", C.c_int), ("loops_total", C.c_int64),
                ("n_failed", C.c_int), ("n_safeguard", C.c_int), ("n_newton", C.c_int),
                ("nnz", C.c_int64), ("entry_evals", C.c_int64), ("cost", C.c_double),
                ("obj", C.c_double), ("err_x", C.c_double), ("ms", C.c_double),
                ("ms_kernel", C.c_double * N_KERNELS), ("ms_start", C.c_double * N_KERNELS),
                ("ms_end", C.c_double * N_KERNELS), ("cells_bin", C.c_int * N_BINS),
                ("evals_bin", C.c_int64 * N_BINS), ("newton_evals", C.c_int64),
                ("newton_mfma_flops", C.c_int64)]

    def as_dict(self):
        return {k: (list(getattr(self, k)) if k in ("ms_kernel", "ms_start", "ms_end", "cells_bin",
                                                     "evals_bin")
                    else getattr(self, k)) for k, _ in self._fields_}


class RunStats(C.Structure):
    _fields_ = [("n_half_iters", C.c_int), ("n_cell_solves", C.c_int),
                ("loops_total", C.c_int64), ("entry_evals", C.c_int64), ("n_failed", C.c_int),
                ("n_safeguard", C.c_int), ("n_newton", C.c_int), ("nnz_max", C.c_int64),
                ("ms_total", C.c_double), ("ms_kernel", C.c_double * N_KERNELS),
                ("launches_bin", C.c_int * N_BINS),
                ("evals_bin", C.c_int64 * N_BINS), ("newton_evals", C.c_int64),
                ("newton_mfma_flops", C.c_int64), ("newton_launches", C.c_int)]

    def as_dict(self):
        return {k: (list(getattr(self, k)) if k in ("ms_kernel", "launches_bin", "evals_bin")
                    else getattr(self, k)) for k, _ in self._fields_}


class TunePoint(C.Structure):
    _fields_ = [("solver_per_cu", C.c_int), ("newton_per_cu", C.c_int), ("stream_wgs", C.c_int),
                ("cells_per_wg", C.c_int), ("ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CostReport(C.Structure):
    _fields_ = [("cost", C.c_double), ("obj", C.c_double), ("err_x", C.c_double),
                ("err_y", C.c_double), ("mass_drift", C.c_double), ("nnz", C.c_int64),
                ("level", C.c_int), ("last_partition", C.c_int), ("eps", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CertReport(C.Structure):
    _fields_ = [("primal", C.c_double), ("dual", C.c_double), ("gap", C.c_double),
                ("rel_gap", C.c_double), ("sum_nu", C.c_double), ("n_uncovered", C.c_int64),
                ("n_edges", C.c_int), ("level", C.c_int), ("eps", C.c_double),
                ("cg_iters", C.c_int), ("cg_rel_resid", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SingleOptions(C.Structure):
    _fields_ = [("err_tol", C.c_double), ("err_norm", C.c_int), ("theta", C.c_double),
                ("absorb", C.c_double), ("max_iter", C.c_int), ("check_every", C.c_int),
                ("cost_p", C.c_double), ("stream", C.c_void_p)]


class SingleReport(C.Structure):
    _fields_ = [("n_stages", C.c_int), ("level", C.c_int), ("eps", C.c_double),
                ("loops_total", C.c_int64), ("loops_max_stage", C.c_int), ("n_absorb", C.c_int),
                ("entries_max", C.c_int64), ("entries_final", C.c_int64),
                ("entry_evals", C.c_int64), ("err_x_l1", C.c_double), ("err_x_linf", C.c_double),
                ("err_y_l1", C.c_double), ("cost", C.c_double), ("primal", C.c_double),
                ("dual", C.c_double), ("plan_mass", C.c_double), ("ms", C.c_double),
                ("failed", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Peaks(C.Structure):
    _fields_ = [("fp32_fma_tflops", C.c_double), ("fp64_fma_tflops", C.c_double),
                ("exp_f32_per_s", C.c_double), ("compute_units", C.c_int),
                ("clock_mhz", C.c_double), ("ms_fp32", C.c_double), ("ms_fp64", C.c_double),
                ("ms_exp", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PlanView(C.Structure):
    _fields_ = [("level", C.c_int), ("H", C.c_int), ("W", C.c_int), ("eps", C.c_double),
                ("n_basic", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p), ("alpha_a", C.c_void_p),
                ("alpha_b", C.c_void_p)]


def _load():
    # PyTorch ships its own HIP runtime.  Loading it first makes the library's
    # dependency on libamdhip64 resolve to that same runtime, so device
    # pointers and streams are shared with torch and only one runtime
    # initialises the GPU in the process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_2001_10986_amd/csrc/build.py`")
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    lib.dd_options_default.argtypes = [P(Options)]
    lib.dd_options_default.restype = None
    lib.dd_init.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int,
                            P(Stage), C.c_int, P(Options), P(C.c_void_p)]
    lib.dd_half_iterate.argtypes = [C.c_void_p, C.c_int, P(IterStats)]
    lib.dd_set_eps.argtypes = [C.c_void_p, C.c_double]
    lib.dd_refine.argtypes = [C.c_void_p]
    lib.dd_run_schedule.argtypes = [C.c_void_p, P(RunStats)]
    lib.dd_cost.argtypes = [C.c_void_p, P(CostReport)]
    lib.dd_single_options_default.argtypes = [P(SingleOptions)]
    lib.dd_single_options_default.restype = None
    lib.dd_single_solve.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int,
                                    C.c_void_p, C.c_int, P(SingleOptions), P(SingleReport),
                                    C.c_void_p, C.c_void_p]
    lib.dd_single_solve.restype = C.c_int
    lib.dd_single_last_error.argtypes = []
    lib.dd_single_last_error.restype = C.c_char_p
    lib.dd_cost_noalloc.argtypes = [C.c_void_p, P(CostReport)]
    lib.dd_certificate.argtypes = [C.c_void_p, P(CertReport), C.c_void_p, C.c_void_p]
    lib.dd_export_plan.argtypes = [C.c_void_p, P(PlanView)]
    lib.dd_import_state.argtypes = [C.c_void_p, P(PlanView)]
    lib.dd_cell_results.argtypes = [C.c_void_p] + [C.c_void_p] * 5
    lib.dd_level_info.argtypes = [C.c_void_p] + [P(C.c_int)] * 6 + [P(C.c_double)]
    lib.dd_free.argtypes = [C.c_void_p]
    lib.dd_free.restype = None
    lib.dd_last_error.argtypes = [C.c_void_p]
    lib.dd_last_error.restype = C.c_char_p
    lib.dd_set_warm_start.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_float]
    lib.dd_set_warm_prediction.argtypes = [C.c_void_p, C.c_void_p, C.c_float]
    lib.dd_set_warm_prediction.restype = C.c_int
    lib.dd_warm_start_count.argtypes = [C.c_void_p, P(C.c_int), P(C.c_longlong)]
    lib.dd_warm_start_count.restype = C.c_int
    lib.dd_collect_cells.argtypes = [C.c_void_p] + [C.c_void_p] * 4 + [C.c_int, P(C.c_int)]
    lib.dd_mlp_get_stream.argtypes = [C.c_void_p]
    lib.dd_mlp_get_stream.restype = C.c_void_p
    lib.dd_batch_create.argtypes = [P(C.c_void_p), C.c_int, C.c_int, P(C.c_void_p)]
    lib.dd_batch_half_iterate.argtypes = [C.c_void_p, C.c_int, P(IterStats)]
    lib.dd_batch_run_schedule.argtypes = [C.c_void_p, P(RunStats)]
    lib.dd_batch_schedule_step.argtypes = [C.c_void_p, P(IterStats), P(C.c_int)]
    lib.dd_set_launch.argtypes = [C.c_void_p, P(TunePoint)]
    lib.dd_batch_set_launch.argtypes = [C.c_void_p, P(TunePoint)]
    lib.dd_get_launch.argtypes = [C.c_void_p, P(TunePoint)]
    lib.dd_get_launch.restype = C.c_int
    for name in ("dd_autotune", "dd_batch_autotune"):
        getattr(lib, name).argtypes = [C.c_void_p, C.c_int, C.c_int, P(TunePoint), P(TunePoint),
                                       C.c_int, P(C.c_int)]
    lib.dd_batch_info.argtypes = [C.c_void_p, P(C.c_int), P(C.c_longlong), P(C.c_int)]
    lib.dd_batch_free.argtypes = [C.c_void_p]
    lib.dd_batch_free.restype = None
    lib.dd_batch_last_error.argtypes = [C.c_void_p]
    lib.dd_batch_last_error.restype = C.c_char_p
    lib.dd_probe_peaks.argtypes = [P(Peaks)]
    lib.dd_probe_peaks.restype = C.c_int
    lib.dd_probe_last_error.argtypes = []
    lib.dd_probe_last_error.restype = C.c_char_p
    for name in ("dd_set_warm_start", "dd_collect_cells", "dd_batch_create",
                 "dd_batch_half_iterate", "dd_batch_run_schedule", "dd_batch_schedule_step",
                 "dd_batch_info", "dd_set_launch", "dd_batch_set_launch", "dd_autotune",
                 "dd_batch_autotune"):
        getattr(lib, name).restype = C.c_int
    for name in ("dd_init", "dd_half_iterate", "dd_set_eps", "dd_refine", "dd_run_schedule",
                 "dd_cost", "dd_export_plan", "dd_import_state", "dd_cell_results",
                 "dd_level_info"):
        getattr(lib, name).restype = C.c_int
    return lib


lib = _load()


class DDError(RuntimeError):
    pass


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _autotune(fn, h, partition, reps, chk):
    best = TunePoint()
    tried = (TunePoint * 32)()
    n = C.c_int()
    chk(fn(h, partition, reps, C.byref(best), tried, 32, C.byref(n)), fn.__name__)
    return best.as_dict(), [tried[i].as_dict() for i in range(min(n.value, 32))]


def probe_peaks():
    """Measured FP32/FP64 multiply-add and FP32 exponential rates of the
    current device (dd_probe_peaks)."""
    out = Peaks()
    st = lib.dd_probe_peaks(C.byref(out))
    if st != 0:
        raise DDError(f"dd_probe_peaks: status {st}: {lib.dd_probe_last_error().decode()}")
    return out.as_dict()


class Problem:
    """One transport problem on the GPU (a dd_ctx).

    mu, nu: H x W float64 arrays (numpy on the host, or torch CUDA tensors,
    which are read in place); schedule: rows (level, eps, n_half_iters).
    """

    def __init__(self, mu, nu, schedule, s=4, n_levels=1, err_tol=1e-5, trunc=1e-15,
                 max_iter=50000, safeguard=1, stream=None, timing=False, accel=1,
                 newton_after=384, precision=DD_PREC_SPLIT, cost_p=2.0, safeguard_after=None):
        # safeguard_after None: 1024 with the Newton fallback, else the loop
        # cap (the plain iteration keeps the safeguard at its cap)
        opt = Options()
        lib.dd_options_default(C.byref(opt))
        opt.err_tol, opt.trunc_threshold = err_tol, trunc
        opt.max_sinkhorn_iter, opt.safeguard = max_iter, safeguard
        opt.timing = 1 if timing else 0
        opt.accel = int(accel)
        opt.newton_after = int(newton_after)
        opt.precision = int(precision)
        opt.cost_p = float(cost_p)
        if safeguard_after is None:
            safeguard_after = 1024 if newton_after > 0 else 0
        opt.safeguard_after = int(safeguard_after)
        on_dev = hasattr(mu, "data_ptr") and getattr(mu, "is_cuda", False)
        if on_dev:
            import torch
            assert mu.dtype == torch.float64 and nu.dtype == torch.float64
            mu_c, nu_c = mu.contiguous(), nu.contiguous()
            self._keep = (mu_c, nu_c)
            H, W = mu_c.shape
            pm, pn = C.c_void_p(mu_c.data_ptr()), C.c_void_p(nu_c.data_ptr())
            opt.inputs_on_device = 1
            if stream is None:
                stream = torch.cuda.current_stream().cuda_stream
        else:
            mu_c = np.ascontiguousarray(mu, dtype=np.float64)
            nu_c = np.ascontiguousarray(nu, dtype=np.float64)
            self._keep = (mu_c, nu_c)
            H, W = mu_c.shape
            pm, pn = _p(mu_c), _p(nu_c)
        opt.stream = stream
        self.H, self.W, self.s, self.n_levels = H, W, s, n_levels
        self.schedule = [tuple(x) for x in schedule]
        arr = (Stage * len(schedule))(*[Stage(int(l), float(e), int(n))
                                        for l, e, n in schedule])
        h = C.c_void_p()
        rc = lib.dd_init(pm, pn, H, W, s, n_levels, arr, len(schedule), C.byref(opt),
                         C.byref(h))
        if rc != 0:
            raise DDError(f"dd_init: {lib.dd_last_error(None).decode()} ({rc})")
        self._h = h

    def _chk(self, rc, what):
        if rc < 0:
            raise DDError(f"{what}: {lib.dd_last_error(self._h).decode()} ({rc})")
        return rc

    def close(self):
        if getattr(self, "_h", None) and lib is not None:
            lib.dd_free(self._h)
        self._h = None

    def __del__(self):
        self.close()

    def half_iterate(self, partition):
        st = IterStats()
        rc = self._chk(lib.dd_half_iterate(self._h, partition, C.byref(st)), "dd_half_iterate")
        d = st.as_dict()
        d["status"] = rc
        return d

    def set_eps(self, eps):
        self._chk(lib.dd_set_eps(self._h, eps), "dd_set_eps")

    def refine(self):
        self._chk(lib.dd_refine(self._h), "dd_refine")

    def run_schedule(self):
        st = RunStats()
        rc = self._chk(lib.dd_run_schedule(self._h, C.byref(st)), "dd_run_schedule")
        d = st.as_dict()
        d["status"] = rc
        return d

    def cost(self):
        r = CostReport()
        self._chk(lib.dd_cost(self._h, C.byref(r)), "dd_cost")
        return r.as_dict()

    def cost_noalloc(self):
        """dd_cost_noalloc: the same report from a static device scratch (no
        device allocation; levels of at most 2^22 pixels)."""
        r = CostReport()
        self._chk(lib.dd_cost_noalloc(self._h, C.byref(r)), "dd_cost_noalloc")
        return r.as_dict()

    def certificate(self, potentials=False):
        """Primal-dual certificate of the current iterate (dd_certificate); with
        potentials=True also the glued alpha_hat and beta_hat (H x W, FP64)."""
        r = CertReport()
        if not potentials:
            rc = self._chk(lib.dd_certificate(self._h, C.byref(r), None, None), "dd_certificate")
            out = r.as_dict()
            out["status"] = rc
            return out
        info = self.level_info()
        H, W = info["H"], info["W"]
        a = np.empty(H * W, dtype=np.float64)
        b = np.empty(H * W, dtype=np.float64)
        rc = self._chk(lib.dd_certificate(self._h, C.byref(r), a.ctypes.data, b.ctypes.data),
                       "dd_certificate")
        out = r.as_dict()
        out["status"] = rc
        out["alpha_hat"], out["beta_hat"] = a.reshape(H, W), b.reshape(H, W)
        return out

    def level_info(self):
        v = [C.c_int() for _ in range(6)]
        e = C.c_double()
        self._chk(lib.dd_level_info(self._h, *[C.byref(x) for x in v], C.byref(e)),
                  "dd_level_info")
        keys = ["level", "H", "W", "n_basic", "n_cells_a", "n_cells_b"]
        out = {k: x.value for k, x in zip(keys, v)}
        out["eps"] = e.value
        return out

    def export(self):
        v = PlanView()
        self._chk(lib.dd_export_plan(self._h, C.byref(v)), "dd_export_plan")
        nb, nnz, H, W = v.n_basic, v.nnz, v.H, v.W
        rp = np.empty(nb + 1, dtype=np.int64)
        col = np.empty(max(nnz, 1), dtype=np.int32)
        val = np.empty(max(nnz, 1), dtype=np.float64)
        aA = np.empty(H * W, dtype=np.float64)
        aB = np.empty(H * W, dtype=np.float64)
        v.row_ptr, v.col, v.val = rp.ctypes.data, col.ctypes.data, val.ctypes.data
        v.alpha_a, v.alpha_b = aA.ctypes.data, aB.ctypes.data
        self._chk(lib.dd_export_plan(self._h, C.byref(v)), "dd_export_plan")
        return {"row_ptr": rp, "col": col[:nnz], "val": val[:nnz], "alpha_a": aA.reshape(H, W),
                "alpha_b": aB.reshape(H, W), "level": v.level, "eps": v.eps}

    def import_state(self, level, eps, row_ptr, col, val, alpha_a, alpha_b):
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        vl = np.ascontiguousarray(val, dtype=np.float64)
        aA = np.ascontiguousarray(alpha_a, dtype=np.float64)
        aB = np.ascontiguousarray(alpha_b, dtype=np.float64)
        v = PlanView()
        v.level, v.eps = level, eps
        v.H, v.W = aA.shape
        v.n_basic = len(rp) - 1
        v.nnz = int(rp[-1])
        v.row_ptr, v.col, v.val = rp.ctypes.data, cl.ctypes.data, vl.ctypes.data
        v.alpha_a, v.alpha_b = aA.ctypes.data, aB.ctypes.data
        self._chk(lib.dd_import_state(self._h, C.byref(v)), "dd_import_state")

    def cell_results(self):
        info = self.level_info()
        last = self.cost()["last_partition"]
        n = info["n_cells_a"] if last == 0 else info["n_cells_b"]
        cost, obj, err = (np.empty(n) for _ in range(3))
        loops, status = np.empty(n, dtype=np.int32), np.empty(n, dtype=np.int32)
        self._chk(lib.dd_cell_results(self._h, _p(cost), _p(obj), _p(err), _p(loops),
                                      _p(status)), "dd_cell_results")
        return {"cost": cost, "obj": obj, "err_x": err, "loops": loops, "status": status}

    def set_launch(self, solver_per_cu=8, newton_per_cu=2, stream_wgs=0, cells_per_wg=0, **_):
        t = TunePoint(solver_per_cu, newton_per_cu, stream_wgs, cells_per_wg, 0.0)
        self._chk(lib.dd_set_launch(self._h, C.byref(t)), "dd_set_launch")

    def get_launch(self):
        t = TunePoint()
        self._chk(lib.dd_get_launch(self._h, C.byref(t)), "dd_get_launch")
        return t.as_dict()

    def autotune(self, partition, reps=1):
        """Time the candidate launch configurations on the next sweep of `partition`
        (state unchanged on return); keeps the fastest.  Returns (best, tried)."""
        return _autotune(lib.dd_autotune, self._h, partition, reps, self._chk)

    def set_warm_start(self, net, policy=1, min_rms=0.0):
        """Attach a warm-start network (paper_2001_10986_amd.mlp.MLP; None detaches).
        policy 1: first sweep of each partition after init/refine/eps change; 2: every
        sweep; a cell takes the prediction if its predicted change has RMS >= min_rms."""
        self._warm_net = net  # keep it alive while attached
        self._chk(lib.dd_set_warm_start(self._h, None if net is None else net.handle,
                                        policy if net is not None else 0, float(min_rms)),
                  "dd_set_warm_start")

    def set_warm_prediction(self, y, min_rms=0.0):
        """dd_set_warm_prediction: apply the rows of the torch CUDA float32
        tensor y (cells of the next sweep's partition x 64, network output
        units) as the start of the next half-iteration only."""
        assert y.is_cuda and y.dtype.itemsize == 4 and y.is_contiguous()
        self._warm_pred = y  # keep it alive until the sweep has run
        self._chk(lib.dd_set_warm_prediction(self._h, C.c_void_p(y.data_ptr()), float(min_rms)),
                  "dd_set_warm_prediction")

    def warm_start_count(self):
        """(sweeps that ran the network, cells that took its start) since init."""
        a, b = C.c_int(), C.c_longlong()
        self._chk(lib.dd_warm_start_count(self._h, C.byref(a), C.byref(b)), "dd_warm_start_count")
        return a.value, b.value

    def collect_cells(self, x, t, m, ids=None):
        """Training samples of the last half-iteration into the torch CUDA tensors
        x (cap x 768), t (cap x 64), m (cap x 64) and optionally ids (cap, int32:
        cell index per row); returns the number of rows."""
        n = C.c_int()
        cap = x.shape[0]
        self._chk(lib.dd_collect_cells(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                       C.c_void_p(m.data_ptr()),
                                       None if ids is None else C.c_void_p(ids.data_ptr()), cap,
                                       C.byref(n)), "dd_collect_cells")
        return n.value

    def basic_marginals(self):
        e = self.export()
        info = self.level_info()
        out = np.zeros((info["n_basic"], info["H"] * info["W"]))
        rp = e["row_ptr"]
        for b in range(info["n_basic"]):
            out[b, e["col"][rp[b]:rp[b + 1]]] = e["val"][rp[b]:rp[b + 1]]
        return out


class Batch:
    """Problems whose sweeps run together (a dd_batch).  The Problems must
    share a stream and outlive the batch; while it exists their own
    half_iterate/run_schedule are refused."""

    def __init__(self, problems, graph=False):
        self.problems = list(problems)
        n = len(self.problems)
        arr = (C.c_void_p * n)(*[p._h for p in self.problems])
        h = C.c_void_p()
        rc = lib.dd_batch_create(arr, n, DD_BATCH_GRAPH if graph else 0, C.byref(h))
        if rc != 0:
            raise DDError(f"dd_batch_create: invalid batch ({rc})")
        self._h = h

    def _chk(self, rc, what):
        if rc < 0:
            raise DDError(f"{what}: {lib.dd_batch_last_error(self._h).decode()} ({rc})")
        return rc

    def close(self):
        if getattr(self, "_h", None) and lib is not None:
            lib.dd_batch_free(self._h)
        self._h = None

    def __del__(self):
        self.close()

    def half_iterate(self, partition):
        n = len(self.problems)
        st = (IterStats * n)()
        rc = self._chk(lib.dd_batch_half_iterate(self._h, partition, st), "dd_batch_half_iterate")
        return [dict(x.as_dict(), status=rc) for x in st]

    def run_schedule(self):
        n = len(self.problems)
        st = (RunStats * n)()
        rc = self._chk(lib.dd_batch_run_schedule(self._h, st), "dd_batch_run_schedule")
        return [dict(x.as_dict(), status=rc) for x in st]

    def set_launch(self, solver_per_cu=8, newton_per_cu=2, stream_wgs=0, cells_per_wg=0, **_):
        t = TunePoint(solver_per_cu, newton_per_cu, stream_wgs, cells_per_wg, 0.0)
        self._chk(lib.dd_batch_set_launch(self._h, C.byref(t)), "dd_batch_set_launch")

    def autotune(self, partition, reps=1):
        return _autotune(lib.dd_batch_autotune, self._h, partition, reps, self._chk)

    def schedule_step(self):
        """One lockstep sweep of the problems' schedules: (problems that ran, stats)."""
        n = len(self.problems)
        st = (IterStats * n)()
        na = C.c_int()
        rc = self._chk(lib.dd_batch_schedule_step(self._h, st, C.byref(na)),
                       "dd_batch_schedule_step")
        return na.value, [dict(x.as_dict(), status=rc) for x in st]

    def info(self):
        a, b, c = C.c_int(), C.c_longlong(), C.c_int()
        self._chk(lib.dd_batch_info(self._h, C.byref(a), C.byref(b), C.byref(c)), "dd_batch_info")
        return {"n_problems": a.value, "n_sweeps": b.value, "n_captures": c.value}


DD_SINGLE_LINF, DD_SINGLE_L1 = 0, 1


def single_solve(mu, nu, schedule, n_levels=1, err_tol=1e-7, err_norm=DD_SINGLE_LINF,
                 theta=1e-10, absorb=30.0, max_iter=200000, check_every=16, cost_p=2.0,
                 potentials=False, stream=None):
    """Single sparse multi-scale Sinkhorn on the whole grid (dd_single_solve,
    include/dd_single.h): host images mu, nu (H x W float64), stages
    (level, eps[, n]).  Returns the report as a dict (status included); with
    potentials=True also the total potentials alpha, beta of the last level."""
    mu_c = np.ascontiguousarray(mu, dtype=np.float64)
    nu_c = np.ascontiguousarray(nu, dtype=np.float64)
    H, W = mu_c.shape
    opt = SingleOptions()
    lib.dd_single_options_default(C.byref(opt))
    opt.err_tol, opt.err_norm, opt.theta, opt.absorb = err_tol, err_norm, theta, absorb
    opt.max_iter, opt.check_every, opt.cost_p = max_iter, check_every, cost_p
    if stream is not None:
        opt.stream = stream
    arr = (Stage * len(schedule))(*[Stage(int(x[0]), float(x[1]), int(x[2]) if len(x) > 2 else 0)
                                    for x in schedule])
    rep = SingleReport()
    lev = max(int(x[0]) for x in schedule)
    f = n_levels - 1 - lev
    a = b = None
    if potentials:
        a = np.empty((H >> f) * (W >> f))
        b = np.empty_like(a)
    rc = lib.dd_single_solve(_p(mu_c), _p(nu_c), H, W, n_levels, arr, len(schedule),
                             C.byref(opt), C.byref(rep), None if a is None else _p(a),
                             None if b is None else _p(b))
    if rc < 0:
        raise DDError(f"dd_single_solve: {lib.dd_single_last_error().decode()} ({rc})")
    out = rep.as_dict()
    out["status"] = rc
    if potentials:
        out["alpha"] = a.reshape(H >> f, W >> f)
        out["beta"] = b.reshape(H >> f, W >> f)
    return out
