"""ctypes binding of librichards.so (include/richards.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Device arrays are torch tensors on the GPU (float64 unless stated); PyTorch
supplies device memory and the stream, nothing else.  If the library has not
been built, or no GPU is present, calls fail loudly: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librichards.so")

OK = 0
EINVAL, ENOMEM, EBUDGET, NONFINITE = -1, -2, -3, -4
LINSOLVE_FAIL, LINESEARCH_FAIL, MAXITER, NOT_SPD, EHIP, ESTATE = -5, -6, -7, -9, -10, -11
STEP_TOO_SMALL = 2
PREC_FP64, PREC_MIXED = 0, 1
WHICH_J, WHICH_A, WHICH_P, WHICH_PT = 0, 1, 2, 3


class RichError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


class Problem(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("hx", C.c_double), ("hy", C.c_double), ("hz", C.c_double),
                ("alpha", C.c_double), ("beta", C.c_double), ("theta_s", C.c_double),
                ("theta_r", C.c_double), ("A", C.c_double), ("gamma", C.c_double),
                ("mean", C.c_int), ("bc_type", C.c_int * 6), ("bc_value", C.c_double * 6),
                ("dt", C.c_double), ("patch_face", C.c_int), ("patch_lo", C.c_double * 2),
                ("patch_hi", C.c_double * 2), ("patch_value", C.c_double), ("mean_vertical", C.c_int)]


class Opts(C.Structure):
    _fields_ = [("fnormtol", C.c_double), ("scsteptol", C.c_double),
                ("max_newton", C.c_int), ("msbset", C.c_int),
                ("ls_alpha", C.c_double), ("mxnewtstep", C.c_double),
                ("gmres_restart", C.c_int), ("eta", C.c_double), ("gmres_maxit", C.c_int),
                ("amg_max_levels", C.c_int), ("amg_coarse_size", C.c_int64),
                ("amg_sweeps", C.c_int), ("coarse_dense_max", C.c_int64),
                ("coarse_l1_sweeps", C.c_int), ("precision", C.c_int), ("gmres_reorth", C.c_double),
                ("aux_dflux", C.c_int), ("amg_refresh", C.c_int), ("amg_smoothed", C.c_int),
                ("tile_kz", C.c_int), ("smoother", C.c_int), ("amg_aggregation", C.c_int),
                ("amg_theta", C.c_double), ("amg_block", C.c_int64),
                ("gmres_block", C.c_int), ("gmres_shift", C.c_double), ("gmres_shift_span", C.c_double)]


class StepStats(C.Structure):
    _fields_ = [("status", C.c_int), ("newton_its", C.c_int), ("jac_builds", C.c_int),
                ("gmres_its", C.c_int), ("ls_backtracks", C.c_int), ("amg_setups", C.c_int),
                ("linsolve_fails", C.c_int), ("levels", C.c_int),
                ("gmres_rounds", C.c_int), ("gmres_redone", C.c_int),
                ("fnorm_inf", C.c_double), ("mass_residual", C.c_double),
                ("min_lambda", C.c_double), ("opc", C.c_double),
                ("t_feval", C.c_double), ("t_jac", C.c_double), ("t_aux", C.c_double),
                ("t_setup", C.c_double), ("t_linsol", C.c_double), ("t_overhead", C.c_double),
                ("t_total", C.c_double), ("bytes_feval", C.c_double), ("bytes_jac", C.c_double),
                ("bytes_linsol", C.c_double), ("bytes_overhead", C.c_double)]


TRACE_TRIALS = 48
EV_ACCEPT, EV_ACCEPT_SHORT, EV_RETRY_GMRES, EV_RETRY_SLOPE, EV_RETRY_LS = 0, 1, 2, 3, 4
EV_FAIL_SLOPE, EV_FAIL_LS, EV_STALL, EV_FAIL_OTHER = 5, 6, 7, 8
RB_NOJ, RB_MSBSET, RB_BIGSTEP, RB_RETRY = 1, 2, 4, 8


class NewtonEvent(C.Structure):
    _fields_ = [("step", C.c_int), ("newton_it", C.c_int), ("since_build", C.c_int), ("reason", C.c_int),
                ("gmres_its", C.c_int), ("gmres_conv", C.c_int), ("truncated", C.c_int), ("outcome", C.c_int),
                ("ntrial", C.c_int), ("nback", C.c_int),
                ("f0", C.c_double), ("slope", C.c_double), ("dnorm2", C.c_double), ("dnorminf", C.c_double),
                ("rel_d", C.c_double), ("mxstep", C.c_double), ("lam", C.c_double), ("f_acc", C.c_double),
                ("step_inf", C.c_double), ("step_rel", C.c_double), ("fnorm_inf", C.c_double),
                ("trial_lam", C.c_double * TRACE_TRIALS), ("trial_f", C.c_double * TRACE_TRIALS)]


def event_dict(e) -> dict:
    d = {f: getattr(e, f) for f, _ in e._fields_ if not f.startswith("trial_")}
    k = min(e.ntrial, TRACE_TRIALS)
    d["trial_lam"] = [e.trial_lam[i] for i in range(k)]
    d["trial_f"] = [e.trial_f[i] for i in range(k)]
    return d


EXPORTS = ["rich_query_bytes", "rich_create", "rich_destroy", "rich_set_state", "rich_get_state",
           "rich_step", "rich_trace_newton", "rich_trace_count", "rich_status_string", "rich_eval_theta", "rich_eval_residual",
           "rich_assemble", "rich_setup_hierarchy", "rich_apply_jacobian", "rich_apply_aux",
           "rich_apply_prec", "rich_gmres", "rich_levels", "rich_level_size", "rich_export_csr",
           "rich_export_aggregates", "rich_match_sweep", "rich_match_sweep_noalloc", "rich_profile", "rich_profile_read",
           "rich_server_create", "rich_server_submit", "rich_server_poll", "rich_server_run_until_idle",
           "rich_server_destroy", "rich_server_set_batching", "rich_server_batch_stats"]

KERNELS = ["spmv_J", "vc0_pre", "vc0_post", "vc0_restrict", "vc1_pre", "vc1_post", "multidot", "update",
           "residual", "block_dot", "block_update"]

_lib = None


def load(path: str = LIB_PATH):
    """Load librichards.so (torch is imported first so the library binds to its HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (one HIP runtime per process: torch's)
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2112_05051_amd.build.build()")
    L = C.CDLL(path)
    P = C.POINTER
    vp, i64p, i32p, dp = C.c_void_p, P(C.c_int64), P(C.c_int32), P(C.c_double)
    L.rich_query_bytes.argtypes = [P(Problem), P(Opts), P(C.c_size_t)]
    L.rich_create.argtypes = [P(Problem), P(Opts), vp, vp, P(vp)]
    L.rich_destroy.argtypes = [vp]
    L.rich_set_state.argtypes = [vp, vp]
    L.rich_get_state.argtypes = [vp, vp]
    L.rich_step.argtypes = [vp, C.c_int, P(StepStats)]
    L.rich_trace_newton.argtypes = [vp, P(NewtonEvent), C.c_int]
    L.rich_trace_count.argtypes = [vp, i64p]
    L.rich_status_string.argtypes = [C.c_int]
    L.rich_status_string.restype = C.c_char_p
    L.rich_eval_theta.argtypes = [vp, vp, vp]
    L.rich_eval_residual.argtypes = [vp, vp, vp, vp]
    L.rich_assemble.argtypes = [vp, vp]
    L.rich_setup_hierarchy.argtypes = [vp]
    L.rich_apply_jacobian.argtypes = [vp, vp, vp]
    L.rich_apply_aux.argtypes = [vp, vp, vp]
    L.rich_apply_prec.argtypes = [vp, vp, vp]
    L.rich_gmres.argtypes = [vp, vp, vp, P(C.c_int), dp]
    L.rich_levels.argtypes = [vp, P(C.c_int)]
    L.rich_level_size.argtypes = [vp, C.c_int, i64p, i64p]
    L.rich_export_csr.argtypes = [vp, C.c_int, C.c_int, i64p, i32p, dp, i64p]
    L.rich_export_aggregates.argtypes = [vp, C.c_int, i32p, i64p]
    L.rich_match_sweep.argtypes = [C.c_int64, vp, vp, vp, vp, i64p, vp]
    L.rich_match_sweep_noalloc.argtypes = [C.c_int64, vp, vp, vp, vp, i64p, vp]
    L.rich_profile.argtypes = [vp, C.c_int]
    L.rich_profile_read.argtypes = [vp, C.c_int, i64p, dp, dp]
    L.rich_server_create.argtypes = [C.c_size_t, C.c_int, vp, P(vp)]
    L.rich_server_submit.argtypes = [vp, P(Problem), P(Opts), dp, dp, C.c_int, i64p]
    L.rich_server_poll.argtypes = [vp, C.c_int64, P(C.c_int), P(C.c_int), dp, P(StepStats), dp, dp]
    L.rich_server_run_until_idle.argtypes = [vp]
    L.rich_server_destroy.argtypes = [vp]
    L.rich_server_set_batching.argtypes = [vp, C.c_int]
    L.rich_server_batch_stats.argtypes = [vp, i64p, i64p]
    for name in EXPORTS:
        getattr(L, name).restype = C.c_int if name != "rich_status_string" else C.c_char_p
    _lib = L
    return L


def status_string(s: int) -> str:
    try:
        return load().rich_status_string(s).decode()
    except Exception:  # library not loadable: still report the number
        return "status"


def _check(rc: int, what: str, ok=(OK,)):
    if rc not in ok:
        raise RichError(rc, what)
    return rc


def make_problem(p) -> Problem:
    """From any object with the rich_problem_t fields (e.g. synth.Problem)."""
    c = Problem()
    for f in ("nx", "ny", "nz", "mean"):
        setattr(c, f, int(getattr(p, f)))
    for f in ("hx", "hy", "hz", "alpha", "beta", "theta_s", "theta_r", "A", "gamma", "dt"):
        setattr(c, f, float(getattr(p, f)))
    for t in range(6):
        c.bc_type[t] = int(p.bc_type[t])
        c.bc_value[t] = float(p.bc_value[t])
    c.patch_face = int(getattr(p, "patch_face", -1))
    for t in range(2):
        c.patch_lo[t] = float(getattr(p, "patch_lo", (0.0, 0.0))[t])
        c.patch_hi[t] = float(getattr(p, "patch_hi", (0.0, 0.0))[t])
    c.patch_value = float(getattr(p, "patch_value", 0.0))
    c.mean_vertical = int(getattr(p, "mean_vertical", -1))
    return c


def make_opts(o) -> Opts:
    c = Opts()
    for f, t in Opts._fields_:
        v = getattr(o, f)
        setattr(c, f, float(v) if t is C.c_double else int(v))
    return c


def _ptr(t, dtype=None):
    import torch
    if not t.is_cuda:
        raise ValueError("device tensor required")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor required")
    return C.c_void_p(t.data_ptr())


def query_bytes(problem, options) -> int:
    L = load()
    b = C.c_size_t()
    _check(L.rich_query_bytes(C.byref(make_problem(problem)), C.byref(make_opts(options)), C.byref(b)),
           "rich_query_bytes")
    return b.value


def stats_dict(s: StepStats) -> dict:
    return {f: getattr(s, f) for f, _ in StepStats._fields_}


class Solver:
    """A device-resident Richards simulation (one rich_handle_t)."""

    def __init__(self, problem, options, Ks, stream=None):
        import torch
        L = load()
        self._L = L
        self.problem, self.options = problem, options
        self.n = int(problem.nx) * int(problem.ny) * int(problem.nz)
        if Ks.numel() != self.n:
            raise ValueError("Ks has the wrong size")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._h = C.c_void_p()
        self._cp, self._co = make_problem(problem), make_opts(options)
        _check(L.rich_create(C.byref(self._cp), C.byref(self._co), _ptr(Ks, torch.float64),
                             C.c_void_p(self.stream.cuda_stream), C.byref(self._h)), "rich_create")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.rich_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _new(self):
        import torch
        return torch.empty(self.n, dtype=torch.float64, device="cuda")

    def set_state(self, p):
        import torch
        _check(self._L.rich_set_state(self._h, _ptr(p, torch.float64)), "rich_set_state")

    def get_state(self):
        p = self._new()
        _check(self._L.rich_get_state(self._h, _ptr(p)), "rich_get_state")
        return p

    def step(self, nsteps: int = 1, raise_on_error: bool = True):
        st = (StepStats * max(1, nsteps))()
        rc = self._L.rich_step(self._h, nsteps, st)
        out = [stats_dict(st[i]) for i in range(nsteps)]
        if raise_on_error and rc < 0:
            raise RichError(rc, "rich_step")
        return out

    def trace(self, capacity: int = 4096):
        """Record the Newton attempts of the following steps (read with events())."""
        self._ev = (NewtonEvent * capacity)()
        _check(self._L.rich_trace_newton(self._h, self._ev, capacity), "rich_trace_newton")

    def events(self) -> list:
        n = C.c_int64()
        _check(self._L.rich_trace_count(self._h, C.byref(n)), "rich_trace_count")
        if n.value > len(self._ev):
            raise RuntimeError("trace capacity exceeded")
        return [event_dict(self._ev[i]) for i in range(n.value)]

    def theta(self, p):
        out = self._new()
        _check(self._L.rich_eval_theta(self._h, _ptr(p), _ptr(out)), "rich_eval_theta")
        return out

    def residual(self, p, theta_old):
        out = self._new()
        _check(self._L.rich_eval_residual(self._h, _ptr(p), _ptr(theta_old), _ptr(out)), "rich_eval_residual")
        return out

    def assemble(self, p):
        _check(self._L.rich_assemble(self._h, _ptr(p)), "rich_assemble")

    def setup_hierarchy(self):
        _check(self._L.rich_setup_hierarchy(self._h), "rich_setup_hierarchy")

    def apply_jacobian(self, x):
        y = self._new()
        _check(self._L.rich_apply_jacobian(self._h, _ptr(x), _ptr(y)), "rich_apply_jacobian")
        return y

    def apply_aux(self, x):
        y = self._new()
        _check(self._L.rich_apply_aux(self._h, _ptr(x), _ptr(y)), "rich_apply_aux")
        return y

    def apply_prec(self, b):
        x = self._new()
        _check(self._L.rich_apply_prec(self._h, _ptr(b), _ptr(x)), "rich_apply_prec")
        return x

    def gmres(self, b):
        x = self._new()
        its, rr = C.c_int(), C.c_double()
        rc = self._L.rich_gmres(self._h, _ptr(b), _ptr(x), C.byref(its), C.byref(rr))
        _check(rc, "rich_gmres", ok=(OK, LINSOLVE_FAIL))
        return x, its.value, rr.value, rc == OK

    def levels(self) -> int:
        n = C.c_int()
        _check(self._L.rich_levels(self._h, C.byref(n)), "rich_levels")
        return n.value

    def level_size(self, level: int):
        n, nnz = C.c_int64(), C.c_int64()
        _check(self._L.rich_level_size(self._h, level, C.byref(n), C.byref(nnz)), "rich_level_size")
        return n.value, nnz.value

    def export_csr(self, which: int, level: int = 0):
        """(indptr int64, indices int32, data float64) numpy arrays."""
        if which in (WHICH_P, WHICH_PT):
            n = self.level_size(level + (which == WHICH_PT))[0]
            nnz = C.c_int64(0)
            dummy = np.empty(1, np.int64)
            st = self._L.rich_export_csr(self._h, which, level, dummy.ctypes.data_as(C.POINTER(C.c_int64)),
                                         dummy.ctypes.data_as(C.POINTER(C.c_int32)),
                                         dummy.ctypes.data_as(C.POINTER(C.c_double)), C.byref(nnz))
            if nnz.value == 0:
                _check(st, "rich_export_csr")
            cap = nnz.value
        elif which == WHICH_J or level == 0:
            n, cap = self.n, 7 * self.n
        else:
            n, cap = self.level_size(level)
        rp = np.empty(n + 1, np.int64)
        col = np.empty(max(cap, 1), np.int32)
        val = np.empty(max(cap, 1), np.float64)
        nnz = C.c_int64(cap)
        _check(self._L.rich_export_csr(self._h, which, level, rp.ctypes.data_as(C.POINTER(C.c_int64)),
                                       col.ctypes.data_as(C.POINTER(C.c_int32)),
                                       val.ctypes.data_as(C.POINTER(C.c_double)), C.byref(nnz)),
               "rich_export_csr")
        return rp, col[:nnz.value], val[:nnz.value]

    def profile(self, enable: bool):
        _check(self._L.rich_profile(self._h, 1 if enable else 0), "rich_profile")

    def profile_read(self) -> dict:
        """{kernel name: (launches, total ms, total algorithmic bytes)}"""
        out = {}
        for k, name in enumerate(KERNELS):
            n, ms, b = C.c_int64(), C.c_double(), C.c_double()
            _check(self._L.rich_profile_read(self._h, k, C.byref(n), C.byref(ms), C.byref(b)), "rich_profile_read")
            out[name] = (n.value, ms.value, b.value)
        return out

    def export_aggregates(self, level: int):
        n, _ = self.level_size(level)
        agg = np.empty(n, np.int32)
        nc = C.c_int64()
        _check(self._L.rich_export_aggregates(self._h, level, agg.ctypes.data_as(C.POINTER(C.c_int32)),
                                              C.byref(nc)), "rich_export_aggregates")
        return agg, nc.value


def match_sweep(rowptr, col, val, stream=None, agg=None, noalloc=False):
    """One pairwise matching sweep on a device CSR matrix -> (agg int32 tensor, n_coarse).

    noalloc: call rich_match_sweep_noalloc (no allocation inside the library;
    agg, when given, is the caller's int32 output tensor of at least n entries)."""
    import torch
    L = load()
    n = rowptr.numel() - 1
    if agg is None:
        agg = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    if agg.numel() < n or agg.dtype != torch.int32:
        raise ValueError("agg must be an int32 tensor of at least n entries")
    nc = C.c_int64()
    s = stream if stream is not None else torch.cuda.current_stream()
    fn, name = (L.rich_match_sweep_noalloc, "rich_match_sweep_noalloc") if noalloc else (L.rich_match_sweep,
                                                                                        "rich_match_sweep")
    _check(fn(n, _ptr(rowptr, torch.int64), _ptr(col, torch.int32), _ptr(val, torch.float64), _ptr(agg),
              C.byref(nc), C.c_void_p(s.cuda_stream)), name)
    return agg[:n], nc.value


REQ_QUEUED, REQ_RUNNING, REQ_DONE = 0, 1, 2
BATCH_OFF, BATCH_FUSED, BATCH_PERSISTENT = 0, 1, 2


class Server:
    """Ensemble server (rich_server_t): FIFO admission by device-memory budget,
    resident simulations on concurrent streams, their preconditioned products
    fused into batched launches when ``fused`` is true (as persistent grids on
    a device work queue when ``persistent`` is also true).  Inputs/outputs are
    host arrays."""

    def __init__(self, hbm_budget_bytes: int, max_active: int = 4, fused: bool = False, stream=None,
                 persistent: bool = False):
        L = load()
        self._L = L
        self._s = C.c_void_p()
        self._n = {}
        self._steps = {}
        hs = C.c_void_p(stream.cuda_stream) if stream is not None else None
        _check(L.rich_server_create(hbm_budget_bytes, max_active, hs, C.byref(self._s)), "rich_server_create")
        mode = BATCH_PERSISTENT if (fused and persistent) else BATCH_FUSED if fused else BATCH_OFF
        _check(L.rich_server_set_batching(self._s, mode), "rich_server_set_batching")

    def batch_stats(self):
        """(flushes, products): batched flushes so far and the products they carried."""
        f, p = C.c_int64(), C.c_int64()
        _check(self._L.rich_server_batch_stats(self._s, C.byref(f), C.byref(p)), "rich_server_batch_stats")
        return f.value, p.value

    def submit(self, problem, options, ks, p0, nsteps: int) -> int:
        ks = np.ascontiguousarray(ks, dtype=np.float64)
        p0 = np.ascontiguousarray(p0, dtype=np.float64)
        rid = C.c_int64()
        cp, co = make_problem(problem), make_opts(options)
        _check(self._L.rich_server_submit(self._s, C.byref(cp), C.byref(co), ks.ctypes.data_as(C.POINTER(C.c_double)),
                                          p0.ctypes.data_as(C.POINTER(C.c_double)), nsteps, C.byref(rid)),
               "rich_server_submit")
        self._n[rid.value] = p0.size
        self._steps[rid.value] = nsteps
        return rid.value

    def poll(self, rid: int):
        """None while queued/running; else a dict with the result."""
        st, res = C.c_int(), C.c_int()
        n, k = self._n[rid], max(1, self._steps[rid])
        p = np.empty(n)
        stats = (StepStats * k)()
        ms = np.empty(k)
        times = np.empty(3)
        _check(self._L.rich_server_poll(self._s, rid, C.byref(st), C.byref(res), p.ctypes.data_as(C.POINTER(C.c_double)),
                                        stats, ms.ctypes.data_as(C.POINTER(C.c_double)),
                                        times.ctypes.data_as(C.POINTER(C.c_double))), "rich_server_poll")
        if st.value != REQ_DONE:
            return None
        nrun = int(times[2])
        return {"status": res.value, "p": p, "stats": [stats_dict(stats[i]) for i in range(nrun)],
                "step_ms": ms[:nrun].copy(), "wait_s": float(times[0]), "run_s": float(times[1])}

    def run_until_idle(self):
        """Block until no request is queued or running."""
        _check(self._L.rich_server_run_until_idle(self._s), "rich_server_run_until_idle")

    def close(self):
        if getattr(self, "_s", None) is not None and self._s.value:
            self._L.rich_server_destroy(self._s)
            self._s = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
