"""ctypes binding of the FP64 CPU oracle (oracle/ddo.c).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the CPU-baseline leg of
the benchmark use it to check the GPU path; the product path never imports it.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


class Opts(C.Structure):
    _fields_ = [("err_tol", C.c_double), ("trunc", C.c_double), ("max_iter", C.c_int),
                ("n_threads", C.c_int), ("safeguard", C.c_int), ("accel", C.c_int),
                ("newton_after", C.c_int), ("cost_p", C.c_double), ("safeguard_after", C.c_int)]


class Stage(C.Structure):
    _fields_ = [("level", C.c_int), ("eps", C.c_double), ("n_half", C.c_int)]


class IterStats(C.Structure):
    _fields_ = [("n_cells", C.c_int), ("loops_total", C.c_int64), ("loops_max", C.c_int),
                ("n_failed", C.c_int), ("n_safeguard", C.c_int), ("n_newton", C.c_int),
                ("nnz", C.c_int64),
                ("cost", C.c_double), ("obj", C.c_double), ("err_x", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CostReport(C.Structure):
    _fields_ = [("cost", C.c_double), ("obj", C.c_double), ("err_x", C.c_double),
                ("err_y", C.c_double), ("mass_drift", C.c_double), ("nnz", C.c_int64),
                ("level", C.c_int), ("last_partition", C.c_int), ("eps", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        _lib = C.CDLL(path)
        P = C.POINTER
        _lib.ddo_init.argtypes = [P(C.c_double), P(C.c_double), C.c_int, C.c_int, C.c_int, C.c_int,
                                  C.c_double, P(Opts), P(C.c_void_p)]
        _lib.ddo_free.argtypes = [C.c_void_p]
        _lib.ddo_free.restype = None
        _lib.ddo_set_eps.argtypes = [C.c_void_p, C.c_double]
        _lib.ddo_half_iterate.argtypes = [C.c_void_p, C.c_int, C.c_void_p, P(IterStats)]
        _lib.ddo_refine.argtypes = [C.c_void_p]
        _lib.ddo_run_schedule.argtypes = [C.c_void_p, P(Stage), C.c_int, P(IterStats)]
        _lib.ddo_cost.argtypes = [C.c_void_p, P(CostReport)]
        _lib.ddo_level_info.argtypes = [C.c_void_p] + [P(C.c_int)] * 6 + [P(C.c_double)] * 2
        _lib.ddo_cells.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
        _lib.ddo_export.argtypes = [C.c_void_p, P(C.c_int64)] + [C.c_void_p] * 5
        _lib.ddo_import.argtypes = [C.c_void_p, C.c_int, C.c_double] + [C.c_void_p] * 5
        _lib.ddo_cell_results.argtypes = [C.c_void_p] + [C.c_void_p] * 5
        _lib.ddo_cell_solve.argtypes = ([C.c_int] + [C.c_void_p] * 3 + [C.c_int] + [C.c_void_p] * 3
                                        + [C.c_double, C.c_double, C.c_int, C.c_int, C.c_int]
                                        + [C.c_void_p] * 5)
        _lib.ddo_cell_solve_p.argtypes = ([C.c_int] + [C.c_void_p] * 3 + [C.c_int]
                                          + [C.c_void_p] * 3
                                          + [C.c_double, C.c_double, C.c_double, C.c_int, C.c_int,
                                             C.c_int] + [C.c_void_p] * 5)
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Oracle:
    """One problem instance of the oracle; mirrors the C-ABI of the GPU library."""

    def __init__(self, mu, nu, s=4, n_levels=1, eps=1.0, err_tol=1e-5, trunc=1e-15,
                 max_iter=50000, n_threads=0, safeguard=1, accel=1, newton_after=384,
                 cost_p=2.0, safeguard_after=None):
        # safeguard_after: loops after which an unconverged cell goes to the
        # safeguard; default 1024 with the Newton fallback, else the loop cap
        # (so that the plain iteration keeps the safeguard at its cap)
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        nu = np.ascontiguousarray(nu, dtype=np.float64)
        assert mu.shape == nu.shape and mu.ndim == 2
        self.H, self.W = mu.shape
        self.s, self.n_levels = s, n_levels
        if safeguard_after is None:
            safeguard_after = 1024 if newton_after > 0 else 0
        o = Opts(err_tol, trunc, max_iter, n_threads, safeguard, accel, newton_after, cost_p,
                 safeguard_after)
        h = C.c_void_p()
        rc = lib().ddo_init(_dp(mu), _dp(nu), self.H, self.W, s, n_levels, eps, C.byref(o),
                            C.byref(h))
        if rc != 0:
            raise ValueError(f"ddo_init failed ({rc})")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ddo_free(self._h)
        self._h = None

    def __del__(self):
        self.close()

    def set_eps(self, eps):
        if lib().ddo_set_eps(self._h, eps) != 0:
            raise ValueError("ddo_set_eps")

    def half_iterate(self, partition, mask=None):
        st = IterStats()
        m = None
        if mask is not None:
            m = np.ascontiguousarray(mask, dtype=np.uint8)
        rc = lib().ddo_half_iterate(self._h, partition, _p(m), C.byref(st))
        if rc < 0:
            raise RuntimeError(f"ddo_half_iterate failed ({rc})")
        return st.as_dict()

    def refine(self):
        rc = lib().ddo_refine(self._h)
        if rc != 0:
            raise RuntimeError(f"ddo_refine failed ({rc})")

    def run_schedule(self, stages):
        arr = (Stage * len(stages))(*[Stage(int(l), float(e), int(n)) for l, e, n in stages])
        st = IterStats()
        rc = lib().ddo_run_schedule(self._h, arr, len(stages), C.byref(st))
        if rc < 0:
            raise RuntimeError(f"ddo_run_schedule failed ({rc})")
        return st.as_dict()

    def cost(self):
        r = CostReport()
        if lib().ddo_cost(self._h, C.byref(r)) != 0:
            raise RuntimeError("ddo_cost")
        return r.as_dict()

    def level_info(self):
        v = [C.c_int() for _ in range(6)]
        d = [C.c_double() for _ in range(2)]
        lib().ddo_level_info(self._h, *[C.byref(x) for x in v], *[C.byref(x) for x in d])
        keys = ["level", "H", "W", "n_basic", "n_cells_a", "n_cells_b"]
        out = {k: x.value for k, x in zip(keys, v)}
        out["eps"], out["h"] = d[0].value, d[1].value
        return out

    def cells(self, partition):
        info = self.level_info()
        n = info["n_cells_a"] if partition == 0 else info["n_cells_b"]
        a = np.empty((n, 4), dtype=np.int32)
        lib().ddo_cells(self._h, partition, _p(a))
        return a

    def export(self):
        info = self.level_info()
        nnz = C.c_int64()
        lib().ddo_export(self._h, C.byref(nnz), None, None, None, None, None)
        rp = np.empty(info["n_basic"] + 1, dtype=np.int64)
        col = np.empty(max(nnz.value, 1), dtype=np.int32)
        val = np.empty(max(nnz.value, 1), dtype=np.float64)
        npx = info["H"] * info["W"]
        aA = np.empty(npx, dtype=np.float64)
        aB = np.empty(npx, dtype=np.float64)
        lib().ddo_export(self._h, C.byref(nnz), _p(rp), _p(col), _p(val), _p(aA), _p(aB))
        n = nnz.value
        return {"row_ptr": rp, "col": col[:n], "val": val[:n],
                "alpha_a": aA.reshape(info["H"], info["W"]),
                "alpha_b": aB.reshape(info["H"], info["W"]), "level": info["level"],
                "eps": info["eps"]}

    def import_state(self, level, eps, row_ptr, col, val, alpha_a, alpha_b):
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        vl = np.ascontiguousarray(val, dtype=np.float64)
        aA = np.ascontiguousarray(alpha_a, dtype=np.float64).ravel()
        aB = np.ascontiguousarray(alpha_b, dtype=np.float64).ravel()
        rc = lib().ddo_import(self._h, level, eps, _p(rp), _p(cl), _p(vl), _p(aA), _p(aB))
        if rc != 0:
            raise ValueError(f"ddo_import failed ({rc})")

    def cell_results(self, partition):
        info = self.level_info()
        n = info["n_cells_a"] if partition == 0 else info["n_cells_b"]
        cost, obj, err = (np.empty(n) for _ in range(3))
        loops, status = np.empty(n, dtype=np.int32), np.empty(n, dtype=np.int32)
        rc = lib().ddo_cell_results(self._h, _p(cost), _p(obj), _p(err), _p(loops), _p(status))
        if rc != 0:
            raise RuntimeError("no half-iteration yet")
        return {"cost": cost, "obj": obj, "err_x": err, "loops": loops, "status": status}

    def basic_marginals(self):
        """Dense (n_basic, H*W) array of the basic-cell Y-marginals."""
        e = self.export()
        info = self.level_info()
        out = np.zeros((info["n_basic"], info["H"] * info["W"]))
        rp = e["row_ptr"]
        for b in range(info["n_basic"]):
            out[b, e["col"][rp[b]:rp[b + 1]]] = e["val"][rp[b]:rp[b + 1]]
        return out


def cell_solve(xr, xc, mu, yr, yc, nu, lam, tol, max_iter, F0=None, accel=0, newton_after=0,
               cost_p=2.0):
    """Solve one cell problem with the oracle's log-domain Sinkhorn (optionally
    accelerated, optionally switching to Newton steps after newton_after loops);
    cost lam * |dx|^cost_p in units of eps."""
    xr = np.ascontiguousarray(xr, dtype=np.int32)
    xc = np.ascontiguousarray(xc, dtype=np.int32)
    yr = np.ascontiguousarray(yr, dtype=np.int32)
    yc = np.ascontiguousarray(yc, dtype=np.int32)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    nu = np.ascontiguousarray(nu, dtype=np.float64)
    nx, ny = len(mu), len(nu)
    F = np.zeros(nx) if F0 is None else np.array(F0, dtype=np.float64)
    G = np.zeros(ny)
    plan = np.zeros((nx, ny))
    loops = C.c_int()
    err = C.c_double()
    rc = lib().ddo_cell_solve_p(nx, _p(xr), _p(xc), _p(mu), ny, _p(yr), _p(yc), _p(nu), lam,
                                cost_p, tol, max_iter, accel, newton_after, _p(F), _p(G),
                                _p(plan), C.byref(loops), C.byref(err))
    if rc < 0:
        raise ValueError(f"ddo_cell_solve failed ({rc})")
    return {"F": F, "G": G, "plan": plan, "loops": loops.value, "err": err.value, "rc": rc & 15,
            "newton": bool(rc & 16)}
