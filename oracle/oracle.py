"""ctypes binding of the plain-C FP64 oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg.  The product library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np
import scipy.sparse as sp

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
OMP_LIB_PATH = os.path.join(HERE, "liboracle_omp.so")  # the same source built with OpenMP (timing only)
SRC = os.path.join(HERE, "oracle.c")

OK, EINVAL, ENOMEM, NONFINITE = 0, -1, -2, -4
LINSOLVE_FAIL, LINESEARCH_FAIL, MAXITER, STEP_TOO_SMALL, NOT_SPD = -5, -6, -7, 2, -9


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2, no fast-math, no FMA contraction),
    and liboracle_omp.so, the same source with OpenMP (per-row loops on all
    host cores, results identical bit for bit; used only for timing)."""
    for path, extra in ((LIB_PATH, []), (OMP_LIB_PATH, ["-fopenmp"])):
        if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
            cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", *extra, SRC, "-o",
                   path + ".tmp", "-lm"]
            subprocess.run(cmd, check=True)
            os.replace(path + ".tmp", path)
    return LIB_PATH


class CProblem(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("hx", C.c_double), ("hy", C.c_double), ("hz", C.c_double),
                ("alpha", C.c_double), ("beta", C.c_double), ("theta_s", C.c_double),
                ("theta_r", C.c_double), ("A", C.c_double), ("gamma", C.c_double),
                ("mean", C.c_int), ("bc_type", C.c_int * 6), ("bc_value", C.c_double * 6),
                ("dt", C.c_double), ("patch_face", C.c_int), ("patch_lo", C.c_double * 2),
                ("patch_hi", C.c_double * 2), ("patch_value", C.c_double), ("mean_vertical", C.c_int)]


class COpts(C.Structure):
    _fields_ = [("fnormtol", C.c_double), ("scsteptol", C.c_double),
                ("max_newton", C.c_int), ("msbset", C.c_int),
                ("ls_alpha", C.c_double), ("mxnewtstep", C.c_double),
                ("gmres_restart", C.c_int), ("eta", C.c_double), ("gmres_maxit", C.c_int),
                ("amg_max_levels", C.c_int), ("amg_coarse_size", C.c_int64),
                ("amg_sweeps", C.c_int), ("coarse_dense_max", C.c_int64),
                ("coarse_l1_sweeps", C.c_int), ("amg_refresh", C.c_int),
                ("aux_dflux", C.c_int), ("amg_smoothed", C.c_int), ("smoother", C.c_int),
                ("amg_aggregation", C.c_int), ("amg_theta", C.c_double), ("amg_block", C.c_int64)]


class CStats(C.Structure):
    _fields_ = [("status", C.c_int), ("newton_its", C.c_int), ("jac_builds", C.c_int),
                ("gmres_its", C.c_int), ("ls_backtracks", C.c_int), ("amg_setups", C.c_int),
                ("linsolve_fails", C.c_int), ("fnorm_inf", C.c_double),
                ("mass_residual", C.c_double), ("min_lambda", C.c_double)]


TRACE_TRIALS = 48
EV_ACCEPT, EV_ACCEPT_SHORT, EV_RETRY_GMRES, EV_RETRY_SLOPE, EV_RETRY_LS = 0, 1, 2, 3, 4
EV_FAIL_SLOPE, EV_FAIL_LS, EV_STALL, EV_FAIL_OTHER = 5, 6, 7, 8
RB_NOJ, RB_MSBSET, RB_BIGSTEP, RB_RETRY = 1, 2, 4, 8


class CEvent(C.Structure):
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


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        # RICH_ORACLE_OMP=1: the OpenMP build (the benchmark's multi-core CPU timing)
        L = C.CDLL(OMP_LIB_PATH if os.environ.get("RICH_ORACLE_OMP") == "1" else LIB_PATH)
        P = C.POINTER
        d, i64, i32 = P(C.c_double), P(C.c_int64), P(C.c_int32)
        vp = C.c_void_p
        L.orc_laws_array.argtypes = [P(CProblem), C.c_int64, d, d, d]
        L.orc_theta.argtypes = [P(CProblem), d, d]
        L.orc_face_mean.argtypes = [P(CProblem), C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, d]
        L.orc_residual.argtypes = [P(CProblem), d, d, d, d]
        L.orc_pattern_nnz.argtypes = [P(CProblem)]
        L.orc_pattern_nnz.restype = C.c_int64
        L.orc_jacobian.argtypes = [P(CProblem), d, d, i64, i32, d]
        L.orc_auxiliary.argtypes = [P(CProblem), d, d, i64, i32, d]
        L.orc_auxiliary_dflux.argtypes = [P(CProblem), d, d, i64, i32, d]
        L.orc_csr_matvec.argtypes = [C.c_int64, i64, i32, d, d, d]
        L.orc_match_sweep.argtypes = [C.c_int64, i64, i32, d, i32]
        L.orc_match_sweep.restype = C.c_int64
        L.orc_galerkin_nnz.argtypes = [C.c_int64, i64, i32, i32, C.c_int64]
        L.orc_galerkin_nnz.restype = C.c_int64
        L.orc_galerkin.argtypes = [C.c_int64, i64, i32, d, i32, C.c_int64, i64, i32, d]
        L.orc_smoothed_prolongator_nnz.argtypes = [C.c_int64, i64, i32, i32, C.c_int64]
        L.orc_smoothed_prolongator_nnz.restype = C.c_int64
        L.orc_smoothed_prolongator.argtypes = [C.c_int64, i64, i32, d, i32, C.c_int64, i64, i32, d]
        L.orc_smoothed_prolongator.restype = C.c_double
        L.orc_rap_nnz.argtypes = [C.c_int64, i64, i32, C.c_int64, i64, i32]
        L.orc_rap_nnz.restype = C.c_int64
        L.orc_rap.argtypes = [C.c_int64, i64, i32, d, C.c_int64, i64, i32, d, i64, i32, d]
        L.orc_vmb_aggregate.argtypes = [C.c_int64, i64, i32, d, C.c_double, C.c_int64, i32]
        L.orc_vmb_aggregate.restype = C.c_int64
        L.orc_greedy_colors.argtypes = [C.c_int64, i64, i32, i32]
        L.orc_mcgs_sweep.argtypes = [C.c_int64, i64, i32, d, i32, C.c_int, C.c_int, d, d]
        L.orc_amg_prolongator_nnz.argtypes = [vp, C.c_int]
        L.orc_amg_prolongator_nnz.restype = C.c_int64
        L.orc_amg_prolongator_export.argtypes = [vp, C.c_int, i64, i32, d]
        L.orc_amg_build.argtypes = [P(COpts), C.c_int64, i64, i32, d, P(vp)]
        L.orc_amg_update_fine.argtypes = [vp, d]
        L.orc_amg_levels.argtypes = [vp]
        L.orc_amg_level_info.argtypes = [vp, C.c_int, i64, i64]
        L.orc_amg_level_export.argtypes = [vp, C.c_int, i64, i32, d, i32]
        L.orc_amg_coarse_is_dense.argtypes = [vp]
        L.orc_amg_apply.argtypes = [vp, d, d]
        L.orc_amg_destroy.argtypes = [vp]
        L.orc_gmres.argtypes = [C.c_int64, i64, i32, d, vp, d, d, C.c_int, C.c_double, C.c_int,
                                P(C.c_int), P(C.c_double)]
        L.orc_solver_create.argtypes = [P(CProblem), P(COpts), d, P(vp)]
        L.orc_solver_step.argtypes = [vp, d, P(CStats)]
        L.orc_solver_destroy.argtypes = [vp]
        L.orc_solver_trace.argtypes = [vp, P(CEvent), C.c_int]
        L.orc_solver_trace_len.argtypes = [vp]
        L.orc_solver_iterate.argtypes = [vp, d]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i64(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _i32(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def cproblem(P) -> CProblem:
    """Convert a synth.Problem (or any object with the same fields)."""
    c = CProblem()
    for f in ("nx", "ny", "nz", "mean"):
        setattr(c, f, int(getattr(P, f)))
    for f in ("hx", "hy", "hz", "alpha", "beta", "theta_s", "theta_r", "A", "gamma", "dt"):
        setattr(c, f, float(getattr(P, f)))
    for t in range(6):
        c.bc_type[t] = int(P.bc_type[t])
        c.bc_value[t] = float(P.bc_value[t])
    c.patch_face = int(getattr(P, "patch_face", -1))
    for t in range(2):
        c.patch_lo[t] = float(getattr(P, "patch_lo", (0.0, 0.0))[t])
        c.patch_hi[t] = float(getattr(P, "patch_hi", (0.0, 0.0))[t])
    c.patch_value = float(getattr(P, "patch_value", 0.0))
    c.mean_vertical = int(getattr(P, "mean_vertical", -1))
    return c


def copts(O) -> COpts:
    c = COpts()
    for f, t in COpts._fields_:
        v = getattr(O, f, 0)
        setattr(c, f, float(v) if t is C.c_double else int(v))
    return c


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def laws(P, p, Ks):
    """(theta, theta', K, K') for every entry of p (eq. s(p), K(p) and their derivatives)."""
    p, Ks = _f64(p), _f64(np.broadcast_to(Ks, np.shape(p)))
    out = np.empty((p.size, 4))
    cp = cproblem(P)
    lib().orc_laws_array(C.byref(cp), p.size, _d(p), _d(Ks), _d(out))
    return out[:, 0], out[:, 1], out[:, 2], out[:, 3]


def face_mean(P, direction, pc, Ksc, pn, Ksn, axis=0):
    """(K_f, dK_f/dp_c, dK_f/dp_n) of one face on the given axis (direction +1: pn on
    the higher-index side)."""
    out = np.empty(3)
    cp = cproblem(P)
    lib().orc_face_mean(C.byref(cp), int(axis), int(direction), float(pc), float(Ksc), float(pn), float(Ksn),
                        _d(out))
    return out[0], out[1], out[2]


def theta(P, p):
    p = _f64(p)
    out = np.empty_like(p)
    cp = cproblem(P)
    lib().orc_theta(C.byref(cp), _d(p), _d(out))
    return out


def residual(P, Ks, p, theta_old):
    Ks, p, theta_old = _f64(Ks), _f64(p), _f64(theta_old)
    out = np.empty_like(p)
    cp = cproblem(P)
    lib().orc_residual(C.byref(cp), _d(Ks), _d(p), _d(theta_old), _d(out))
    return out


def _assemble(fn, P, Ks, p):
    Ks, p = _f64(Ks), _f64(p)
    cp = cproblem(P)
    n = p.size
    nnz = lib().orc_pattern_nnz(C.byref(cp))
    rp = np.empty(n + 1, np.int64)
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz)
    fn(C.byref(cp), _d(Ks), _d(p), _i64(rp), _i32(col), _d(val))
    return sp.csr_matrix((val, col, rp), shape=(n, n))


def jacobian(P, Ks, p):
    """Analytic Jacobian of the residual as a scipy CSR matrix (7-point pattern)."""
    return _assemble(lib().orc_jacobian, P, Ks, p)


def auxiliary(P, Ks, p, dflux=False):
    """Diffusion-only preconditioner matrix (symmetric M-matrix) as scipy CSR;
    dflux adds the flux-derivative terms of the diffusion Jacobian to its diagonal."""
    return _assemble(lib().orc_auxiliary_dflux if dflux else lib().orc_auxiliary, P, Ks, p)


def _csr_parts(A):
    A = sp.csr_matrix(A)
    return (np.ascontiguousarray(A.indptr, np.int64), np.ascontiguousarray(A.indices, np.int32),
            _f64(A.data))


def match_sweep(A):
    rp, col, val = _csr_parts(A)
    agg = np.empty(A.shape[0], np.int32)
    nc = lib().orc_match_sweep(A.shape[0], _i64(rp), _i32(col), _d(val), _i32(agg))
    return agg, int(nc)


def galerkin(A, agg, nc):
    rp, col, val = _csr_parts(A)
    agg = np.ascontiguousarray(agg, np.int32)
    n = A.shape[0]
    nnz = lib().orc_galerkin_nnz(n, _i64(rp), _i32(col), _i32(agg), nc)
    crp = np.empty(nc + 1, np.int64)
    ccol = np.empty(nnz, np.int32)
    cval = np.empty(nnz)
    lib().orc_galerkin(n, _i64(rp), _i32(col), _d(val), _i32(agg), nc, _i64(crp), _i32(ccol), _d(cval))
    return sp.csr_matrix((cval, ccol, crp), shape=(nc, nc))


def smoothed_prolongator(A, agg, nc):
    """P = (I - omega D^{-1} A) P_t for the aggregates agg; returns (P, omega)."""
    rp, col, val = _csr_parts(A)
    agg = np.ascontiguousarray(agg, np.int32)
    n = A.shape[0]
    nnz = lib().orc_smoothed_prolongator_nnz(n, _i64(rp), _i32(col), _i32(agg), nc)
    prow = np.empty(n + 1, np.int64)
    pcol = np.empty(nnz, np.int32)
    pval = np.empty(nnz)
    omega = lib().orc_smoothed_prolongator(n, _i64(rp), _i32(col), _d(val), _i32(agg), nc, _i64(prow),
                                           _i32(pcol), _d(pval))
    return sp.csr_matrix((pval, pcol, prow), shape=(n, nc)), float(omega)


def vmb_aggregate(A, theta, block):
    """Decoupled greedy aggregation of A (blocks of `block` rows); returns (agg, number of aggregates)."""
    rp, col, val = _csr_parts(A)
    agg = np.empty(A.shape[0], np.int32)
    nc = lib().orc_vmb_aggregate(A.shape[0], _i64(rp), _i32(col), _d(val), float(theta), int(block), _i32(agg))
    return agg, int(nc)


def greedy_colors(A):
    """Greedy colouring of A's graph in index order; returns (colour array, number of colours)."""
    rp, col, _ = _csr_parts(A)
    color = np.empty(A.shape[0], np.int32)
    nc = lib().orc_greedy_colors(A.shape[0], _i64(rp), _i32(col), _i32(color))
    return color, int(nc)


def mcgs_sweep(A, color, ncolor, direction, b, x):
    """One multicolour Gauss-Seidel sweep on A x = b from x (forward: direction +1,
    colours ascending; backward: -1); returns the new x."""
    rp, col, val = _csr_parts(A)
    x = np.array(x, dtype=np.float64)
    lib().orc_mcgs_sweep(A.shape[0], _i64(rp), _i32(col), _d(val), _i32(np.asarray(color, np.int32)),
                         int(ncolor), int(direction), _d(_f64(b)), _d(x))
    return x


def rap(A, P):
    """C = P^T (A P) with the oracle's summation order."""
    rp, col, val = _csr_parts(A)
    P = sp.csr_matrix(P)
    prow, pcol, pval = _csr_parts(P)
    n, nc = P.shape
    nnz = lib().orc_rap_nnz(n, _i64(rp), _i32(col), nc, _i64(prow), _i32(pcol))
    crow = np.empty(nc + 1, np.int64)
    ccol = np.empty(nnz, np.int32)
    cval = np.empty(nnz)
    lib().orc_rap(n, _i64(rp), _i32(col), _d(val), nc, _i64(prow), _i32(pcol), _d(pval), _i64(crow),
                  _i32(ccol), _d(cval))
    return sp.csr_matrix((cval, ccol, crow), shape=(nc, nc))


class AMG:
    """Oracle AMG hierarchy built from a fine matrix (keeps its own copies)."""

    def __init__(self, opts, A):
        self._h = C.c_void_p()
        self._parts = _csr_parts(A)
        rp, col, val = self._parts
        co = copts(opts)
        rc = lib().orc_amg_build(C.byref(co), A.shape[0], _i64(rp), _i32(col), _d(val), C.byref(self._h))
        if rc != OK:
            raise RuntimeError(f"orc_amg_build failed: {rc}")
        self.n = A.shape[0]

    def update_fine(self, A):
        val = _f64(sp.csr_matrix(A).data)
        rc = lib().orc_amg_update_fine(self._h, _d(val))
        if rc != OK:
            raise RuntimeError(f"orc_amg_update_fine failed: {rc}")

    @property
    def levels(self) -> int:
        return lib().orc_amg_levels(self._h)

    @property
    def coarse_dense(self) -> bool:
        return bool(lib().orc_amg_coarse_is_dense(self._h))

    def level(self, l):
        n, nnz = C.c_int64(), C.c_int64()
        lib().orc_amg_level_info(self._h, l, C.byref(n), C.byref(nnz))
        rp = np.empty(n.value + 1, np.int64)
        col = np.empty(nnz.value, np.int32)
        val = np.empty(nnz.value)
        agg = np.empty(n.value, np.int32) if l < self.levels - 1 else None
        lib().orc_amg_level_export(self._h, l, _i64(rp), _i32(col), _d(val),
                                   _i32(agg) if agg is not None else None)
        return sp.csr_matrix((val, col, rp), shape=(n.value, n.value)), agg

    def prolongator(self, l):
        """The smoothed prolongator of level l (None for piecewise-constant hierarchies)."""
        nnz = lib().orc_amg_prolongator_nnz(self._h, l)
        if nnz == 0:
            return None
        n = self.level(l)[0].shape[0]
        nc = self.level(l + 1)[0].shape[0]
        prow = np.empty(n + 1, np.int64)
        pcol = np.empty(nnz, np.int32)
        pval = np.empty(nnz)
        lib().orc_amg_prolongator_export(self._h, l, _i64(prow), _i32(pcol), _d(pval))
        return sp.csr_matrix((pval, pcol, prow), shape=(n, nc))

    def apply(self, b):
        b = _f64(b)
        x = np.empty_like(b)
        lib().orc_amg_apply(self._h, _d(b), _d(x))
        return x

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.orc_amg_destroy(self._h)
            self._h = C.c_void_p()


def gmres(J, b, amg: AMG | None = None, restart=30, eta=1e-6, maxit=200):
    rp, col, val = _csr_parts(J)
    b = _f64(b)
    x = np.empty_like(b)
    its, rr = C.c_int(), C.c_double()
    conv = lib().orc_gmres(J.shape[0], _i64(rp), _i32(col), _d(val), amg._h if amg else None,
                           _d(b), _d(x), restart, eta, maxit, C.byref(its), C.byref(rr))
    return x, bool(conv), its.value, rr.value


def stats_dict(s: CStats) -> dict:
    return {f: getattr(s, f) for f, _ in CStats._fields_}


class Solver:
    """Time-stepping oracle: backward Euler + modified inexact Newton + AMG-GMRES."""

    def __init__(self, P, opts, Ks):
        self._h = C.c_void_p()
        self.P, self.opts = P, opts
        self._cp, self._co = cproblem(P), copts(opts)
        Ks = _f64(Ks)
        rc = lib().orc_solver_create(C.byref(self._cp), C.byref(self._co), _d(Ks), C.byref(self._h))
        if rc != OK:
            raise RuntimeError(f"orc_solver_create failed: {rc}")

    def step(self, p):
        """Advance p (float64 array, updated in place) by one time step; returns stats."""
        assert p.dtype == np.float64 and p.flags.c_contiguous
        st = CStats()
        lib().orc_solver_step(self._h, _d(p), C.byref(st))
        return stats_dict(st)

    def trace(self, capacity: int = 4096):
        """Record the Newton attempts of the following steps (read with events())."""
        self._ev = (CEvent * capacity)()
        lib().orc_solver_trace(self._h, self._ev, capacity)

    def iterate(self, n):
        """The last Newton iterate of the most recent step (n values)."""
        u = np.empty(n)
        lib().orc_solver_iterate(self._h, _d(u))
        return u

    def events(self) -> list:
        n = lib().orc_solver_trace_len(self._h)
        assert n <= len(self._ev), "trace capacity exceeded"
        return [event_dict(self._ev[i]) for i in range(n)]

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.orc_solver_destroy(self._h)
            self._h = C.c_void_p()
