"""Pins of the oracle's Newton controller (Section 3) through its per-attempt record.

Every attempt of the modified inexact Newton method (rebuild test, GMRES
solve, line search) is recorded by the oracle.  The checks below recompute,
independently of the oracle's code, what the method prescribes at each
recorded decision:

- the Armijo condition f(u + lam d) <= f0 + alpha lam slope at every accepted
  step, with f = 0.5 ||Phi||_2^2 re-evaluated from the residual (itself pinned
  elsewhere) at the returned states;
- every backtracking step: the minimiser of the quadratic (first reduction) or
  cubic (later ones) model of f along d through the recorded values, found
  with numpy's linear solver and polynomial roots, then kept in
  [0.1 lam, 0.5 lam] (Dennis & Schnabel, Algorithm A6.3.1, the published
  method behind the paper's Armijo-Goldstein search);
- the lengthening of a full step while the beta condition holds;
- the rebuild schedule of eq. (jacobian_update_condition): the iteration
  counter persisting across time steps, the step-length rule, the retries;
- the outcome of every attempt (retry with a stale J, failure with a fresh
  one, short-step stall) and the per-step counters.

The workloads are small rough-field requests whose option variants drive the
controller through each branch: backtracking with cubic models, stale-J
GMRES failures, line-search failures, truncated steps, beta lengthening and
short-step stalls.
"""
import math

import numpy as np
import pytest

import synth

BETA = 0.9


def _variant_runs(orc):
    """(options variant, request index) -> (recipe, per-step stats, events, states)."""
    variants = {
        "base": {},
        "gmres8": dict(gmres_maxit=8),
        "msbset3": dict(msbset=3),
        "truncated": dict(mxnewtstep=20.0),
        "onestep": dict(gmres_maxit=1, eta=0.99),
    }
    runs = {}
    for vname, kw in variants.items():
        reqs = synth.serving_stream(count=40, sizes=(12,), nsteps=3)
        for idx in (0, 12, 19, 36):
            _, r = reqs[idx]
            r.options.precision = synth.FP64
            r.options.max_newton = 40
            for k, v in kw.items():
                setattr(r.options, k, v)
            ks = r.ks()
            o = orc.Solver(r.problem, r.options, ks)
            o.trace(20000)
            p = r.p0().copy()
            states, stats = [p.copy()], []
            for _ in range(r.nsteps):
                st = o.step(p)
                stats.append(st)
                states.append(p.copy())
                if st["status"] < 0:
                    break
            runs[(vname, idx)] = (r, ks, stats, o.events(), states)
    return runs


@pytest.fixture(scope="module")
def runs(orc):
    return _variant_runs(orc)


def _accepted(e, orc):
    return e["outcome"] in (orc.EV_ACCEPT, orc.EV_ACCEPT_SHORT, orc.EV_STALL)


def test_branch_coverage(runs, orc):
    """The workloads reach every branch the pins below are about."""
    outcomes, reasons = set(), 0
    cubic = beta = nontrunc = trunc = 0
    for r, ks, stats, ev, _ in runs.values():
        for e in ev:
            outcomes.add(e["outcome"])
            reasons |= e["reason"]
            cubic += max(0, e["nback"] - 1)
            beta += e["ntrial"] - e["nback"] - 1 if _accepted(e, orc) else 0
            trunc += e["truncated"]
            nontrunc += not e["truncated"]
    assert {orc.EV_ACCEPT, orc.EV_ACCEPT_SHORT, orc.EV_RETRY_GMRES, orc.EV_RETRY_LS, orc.EV_FAIL_LS,
            orc.EV_STALL} <= outcomes
    assert reasons == orc.RB_NOJ | orc.RB_MSBSET | orc.RB_BIGSTEP | orc.RB_RETRY
    assert cubic > 50 and beta > 3 and trunc > 50 and nontrunc > 50


def test_counters_are_sums_of_attempts(runs, orc):
    for key, (r, ks, stats, ev, _) in runs.items():
        for s, st in enumerate(stats):
            es = [e for e in ev if e["step"] == s]
            assert st["newton_its"] == sum(_accepted(e, orc) for e in es), key
            assert st["jac_builds"] == sum(e["reason"] != 0 for e in es), key
            assert st["ls_backtracks"] == sum(e["nback"] for e in es), key
            assert st["gmres_its"] == sum(e["gmres_its"] for e in es), key
            assert st["linsolve_fails"] == sum(not e["gmres_conv"] for e in es if e["outcome"] != orc.EV_FAIL_OTHER), key


def test_armijo_and_residual_at_returned_states(runs, orc):
    """Every accepted step meets the Armijo condition; f0 of an attempt is the
    previous accepted f; the recorded f values agree with 0.5 ||Phi||^2
    recomputed from the returned states."""
    for key, (r, ks, stats, ev, states) in runs.items():
        P, alpha = r.problem, r.options.ls_alpha
        for s, st in enumerate(stats):
            es = [e for e in ev if e["step"] == s]
            th = orc.theta(P, states[s])
            F0 = orc.residual(P, ks, states[s], th)
            f = 0.5 * float(F0 @ F0)
            if es:
                assert math.isclose(es[0]["f0"], f, rel_tol=1e-12), key
                f = es[0]["f0"]
            for e in es:
                assert e["f0"] == f, key
                if _accepted(e, orc):
                    assert e["f_acc"] <= e["f0"] + alpha * e["lam"] * e["slope"], key
                    assert e["slope"] < 0 and 0 < e["lam"]
                    f = e["f_acc"]
            if st["status"] >= 0:
                F1 = orc.residual(P, ks, states[s + 1], th)
                assert math.isclose(0.5 * float(F1 @ F1), f, rel_tol=1e-12, abs_tol=1e-300), key
                assert np.abs(F1).max() == pytest.approx(st["fnorm_inf"], rel=1e-12)


def _quadratic_min(f0, slope, lam, fl):
    """Minimiser of q(x) = c0 + c1 x + c2 x^2 with q(0) = f0, q'(0) = slope, q(lam) = fl."""
    A = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [1.0, lam, lam * lam]])
    c0, c1, c2 = np.linalg.solve(A, np.array([f0, slope, fl]))
    assert c2 > 0  # Armijo failed at lam, so the parabola turns upward
    return -c1 / (2.0 * c2)


def _cubic_min(f0, slope, lp, fp, lam, fl):
    """Local minimiser (smallest positive) of the cubic c with c(0) = f0, c'(0) = slope
    through (lp, fp) and (lam, fl); None if it has none."""
    A = np.array([[1.0, 0, 0, 0], [0, 1.0, 0, 0], [1.0, lp, lp ** 2, lp ** 3], [1.0, lam, lam ** 2, lam ** 3]])
    c = np.linalg.solve(A, np.array([f0, slope, fp, fl]))
    if abs(c[3]) < 1e-14 * max(abs(c[2]), 1e-300) * max(lam, 1e-300) ** -1:
        return -c[1] / (2.0 * c[2]) if c[2] > 0 else None
    roots = np.roots([3.0 * c[3], 2.0 * c[2], c[1]])
    mins = [x.real for x in roots if abs(x.imag) <= 1e-12 * abs(x) and 2.0 * c[2] + 6.0 * c[3] * x.real > 0]
    return min(mins) if mins else None


def test_backtracking_steps_are_model_minimisers(runs, orc):
    checked = {"quad": 0, "cubic": 0, "clamped": 0}
    for key, (r, ks, stats, ev, _) in runs.items():
        alpha, tol = r.options.ls_alpha, r.options.scsteptol
        for e in ev:
            lam, fval = e["trial_lam"], e["trial_f"]
            nb = e["nback"]
            if e["ntrial"] == 0 or e["ntrial"] > len(lam):
                continue
            assert lam[0] == 1.0
            lam_min = tol / e["rel_d"] if e["rel_d"] > 0 else 0.0
            last_finite = None
            for k in range(nb):
                lk, fk = lam[k], fval[k]
                # a backtracking trial failed Armijo and was not below the minimum step
                assert not (math.isfinite(fk) and fk <= e["f0"] + alpha * lk * e["slope"]), key
                assert lk >= lam_min, key
                nxt = lam[k + 1]
                assert 0.1 * lk * (1 - 1e-15) <= nxt <= 0.5 * lk * (1 + 1e-15), key
                if not math.isfinite(fk):
                    assert nxt == pytest.approx(0.1 * lk, rel=1e-15)
                    continue
                if last_finite is None:
                    model = _quadratic_min(e["f0"], e["slope"], lk, fk)
                    kind = "quad"
                else:
                    model = _cubic_min(e["f0"], e["slope"], last_finite[0], last_finite[1], lk, fk)
                    kind = "cubic"
                last_finite = (lk, fk)
                want = 0.5 * lk if model is None else min(max(model, 0.1 * lk), 0.5 * lk)
                if model is not None and 0.1 * lk < model < 0.5 * lk:
                    checked[kind] += 1
                else:
                    checked["clamped"] += 1
                assert nxt == pytest.approx(want, rel=1e-7, abs=1e-12 * lk), (key, k, kind)
            if e["outcome"] in (orc.EV_RETRY_LS, orc.EV_FAIL_LS):
                # failure: the last trial failed Armijo below the minimum step
                assert e["ntrial"] == nb + 1
                lk, fk = lam[nb], fval[nb]
                assert lk < lam_min and not (math.isfinite(fk) and fk <= e["f0"] + alpha * lk * e["slope"])
    assert checked["quad"] > 20 and checked["cubic"] > 20 and checked["clamped"] > 20, checked


def test_beta_condition_lengthens_full_steps(runs, orc):
    lengthened = 0
    for key, (r, ks, stats, ev, _) in runs.items():
        alpha = r.options.ls_alpha
        for e in ev:
            if not _accepted(e, orc) or e["ntrial"] > len(e["trial_lam"]):
                continue
            nb = e["nback"]
            ext_lam, ext_f = e["trial_lam"][nb + 1:], e["trial_f"][nb + 1:]
            lam, f = e["trial_lam"][nb], e["trial_f"][nb]
            if nb > 0 or e["truncated"]:
                assert not ext_lam and e["lam"] == lam, key
                continue
            # lengthening continues while the beta condition fails to hold ... (Section 3)
            for lt, ft in zip(ext_lam, ext_f):
                assert f < e["f0"] + BETA * lam * e["slope"] and lt == 2.0 * lam
                assert 2.0 * lam * e["dnorm2"] <= e["mxstep"] * (1 + 1e-12)
                if not (math.isfinite(ft) and ft <= e["f0"] + alpha * lt * e["slope"]):
                    break
                lam, f = lt, ft
                lengthened += 1
            else:
                stop = (f >= e["f0"] + BETA * lam * e["slope"] or 2.0 * lam * e["dnorm2"] > e["mxstep"]
                        or len(ext_lam) == 10)
                assert stop, key
            assert e["lam"] == lam and e["f_acc"] == f, key
    assert lengthened > 3


def test_rebuild_schedule_follows_jacobian_update_condition(runs, orc):
    """Rebuild at an attempt iff no J exists yet, msbset accepted iterations have
    passed since the last rebuild (the counter persisting across time steps),
    the previous accepted step of this time step had ||lam d||_inf > 1.5, or
    the previous attempt asked for a retry."""
    for key, (r, ks, stats, ev, _) in runs.items():
        msbset, tol = r.options.msbset, r.options.scsteptol
        have_j, since = False, 0
        cur_step, prev_step, retry = -1, 0.0, False
        for e in ev:
            if e["step"] != cur_step:
                cur_step, prev_step, retry = e["step"], 0.0, False
            want = ((0 if have_j else orc.RB_NOJ) | (orc.RB_MSBSET if have_j and since >= msbset else 0)
                    | (orc.RB_BIGSTEP if prev_step > 1.5 else 0) | (orc.RB_RETRY if retry else 0))
            assert e["since_build"] == since and e["reason"] == want, (key, e["step"], e["newton_it"])
            fresh = want != 0
            if fresh:
                have_j, since, retry = True, 0, False
            # outcome of the attempt, from its recorded numbers
            if not e["gmres_conv"] and not fresh:
                assert e["outcome"] == orc.EV_RETRY_GMRES
                retry = True
                continue
            if e["outcome"] == orc.EV_FAIL_OTHER:
                break
            assert e["truncated"] == (e["dnorm2"] >= e["mxstep"] * (1 - 1e-12))
            if not e["slope"] < 0:
                assert e["outcome"] == (orc.EV_RETRY_SLOPE if not fresh else orc.EV_FAIL_SLOPE)
                retry = not fresh
                continue
            if e["outcome"] in (orc.EV_RETRY_LS, orc.EV_FAIL_LS):
                assert e["outcome"] == (orc.EV_RETRY_LS if not fresh else orc.EV_FAIL_LS)
                retry = not fresh
                continue
            since += 1
            assert e["step_inf"] == pytest.approx(e["lam"] * e["dnorminf"], rel=1e-15)
            if e["fnorm_inf"] <= r.options.fnormtol:
                assert e["outcome"] == orc.EV_ACCEPT
                continue
            if e["step_rel"] < tol:
                assert e["outcome"] == (orc.EV_ACCEPT_SHORT if not fresh else orc.EV_STALL)
                retry = not fresh
            else:
                assert e["outcome"] == orc.EV_ACCEPT
            prev_step = e["step_inf"]
