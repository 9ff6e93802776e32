"""The GPU's Newton controller against the oracle's, attempt by attempt.

Both sides record every attempt of the modified inexact Newton method
(Section 3): the rebuild test of eq. (jacobian_update_condition), the GMRES
solve and the line search.  In FP64 the two records must agree: the same
attempts with the same rebuild reasons and outcomes, the same number of
backtracking and lengthening trials, GMRES iterations within one per solve
(classical vs modified Gram-Schmidt), and the same accepted steps up to the
difference of two eta-accurate linear solves.  The per-step counters
(Newton iterations, Jacobian builds, backtracks) must be equal.

The workloads are the small rough-field requests and option variants whose
oracle records are pinned on the CPU (tests/test_oracle_newton.py): they
cover backtracking with quadratic and cubic models, stale-J GMRES and
line-search failures, truncated steps, full-step lengthening and runs that
end at the Newton iteration limit.
"""
import numpy as np
import pytest

import synth
from tests.helpers import smooth_recipe

pytestmark = pytest.mark.gpu

VARIANTS = {
    "base": {},
    "gmres8": dict(gmres_maxit=8),
    "msbset3": dict(msbset=3),
    "truncated": dict(mxnewtstep=20.0),
    "onestep": dict(gmres_maxit=1, eta=0.99),
    "block1": dict(gmres_block=1),
}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def rich():
    import paper_2112_05051_amd as r
    r.load()
    return r


def _run_both(rich, torch, orc, rec, nsteps):
    P, opts = rec.problem, rec.options
    ks, p0 = rec.ks(), rec.p0()
    s = rich.Solver(P, opts, torch.from_numpy(ks).to("cuda"))
    s.set_state(torch.from_numpy(p0).to("cuda"))
    s.trace(20000)
    o = orc.Solver(P, opts, ks)
    o.trace(20000)
    po = p0.copy()
    out = []
    for _ in range(nsteps):
        sg = s.step(1, raise_on_error=False)[0]
        so = o.step(po)
        out.append((sg, so, s.get_state().cpu().numpy(), po.copy()))
        if sg["status"] < 0 or so["status"] < 0:
            break
    return out, s.events(), o.events()


def _compare_events(eg, eo, what):
    """Same attempts, decisions and trial counts; numbers within what two
    eta-accurate solves of the same system allow.  Values of f = 0.5 ||Phi||^2
    are compared relative to the step's initial f (near convergence they are
    set by the GMRES residual, itself known to eta only)."""
    assert len(eg) == len(eo), (what, len(eg), len(eo))
    fscale = {}
    for o in eo:
        fscale.setdefault(o["step"], o["f0"])
    for k, (g, o) in enumerate(zip(eg, eo)):
        where = (what, k, o["step"], o["newton_it"])
        for f in ("step", "newton_it", "since_build", "reason", "outcome", "truncated", "nback", "ntrial",
                  "gmres_conv"):
            assert g[f] == o[f], (where, f, g[f], o[f])
        assert abs(g["gmres_its"] - o["gmres_its"]) <= 1, (where, g["gmres_its"], o["gmres_its"])
        fabs = 1e-9 * fscale[o["step"]]
        for f in ("f0", "f_acc"):
            assert g[f] == pytest.approx(o[f], rel=1e-4, abs=fabs), (where, f, g[f], o[f])
        for fg, fo in zip(g["trial_f"], o["trial_f"]):
            assert fg == pytest.approx(fo, rel=1e-4, abs=fabs), (where, "trial_f")
        assert g["slope"] == pytest.approx(o["slope"], rel=1e-4, abs=2e-6 * fscale[o["step"]]), (where, "slope")
        for f in ("dnorm2", "lam"):
            assert g[f] == pytest.approx(o[f], rel=1e-4, abs=1e-12), (where, f, g[f], o[f])
        for lg, lo in zip(g["trial_lam"], o["trial_lam"]):
            assert lg == pytest.approx(lo, rel=1e-4), (where, "trial_lam")


def _compare_counters(out):
    for s, (sg, so, pg, po) in enumerate(out):
        assert sg["status"] == so["status"], (s, sg["status"], so["status"])
        for f in ("newton_its", "jac_builds", "ls_backtracks", "amg_setups", "linsolve_fails"):
            assert sg[f] == so[f], (s, f, sg[f], so[f])


# On some runs that never converge the two iterations drift apart after many
# attempts (rounding differences of the two residual codes grow through
# hundreds of upstream switches) and there is no single record to compare;
# the runs below keep one record to the end.  The branches that only such
# long failing runs reach (stalls, line-search failure with a fresh J) are
# pinned on the CPU.  Request 12 amplifies the differences of the two linear
# solves about tenfold every three attempts from its 18th attempt on, up to
# its 36th: its record stays within 1e-4 to the end only where the solves
# agree with the oracle's to about 1e-12 (one-vector rounds: 7e-5 at the
# peak), not with s-step rounds, whose solves agree to 1e-11..1e-10 -- far
# inside eta, but enough to change a rebuild decision by the 30th attempt.
# It runs with one-vector rounds; the s-step rounds are compared on the
# other records.
@pytest.mark.parametrize("variant,idx", [("block1", 12), ("base", 19), ("gmres8", 0), ("gmres8", 10),
                                         ("truncated", 0), ("onestep", 1)])
def test_newton_record_matches_oracle(rich, torch, orc, variant, idx):
    _, rec = synth.serving_stream(count=40, sizes=(12,), nsteps=3)[idx]
    rec.options.precision = synth.FP64
    rec.options.max_newton = 40
    for k, v in VARIANTS[variant].items():
        setattr(rec.options, k, v)
    out, eg, eo = _run_both(rich, torch, orc, rec, rec.nsteps)
    _compare_counters(out)
    _compare_events(eg, eo, (variant, idx))
    for sg, so, pg, po in out:
        if sg["status"] >= 0:
            assert np.linalg.norm(pg - po) <= 1e-6 * np.linalg.norm(po)


@pytest.mark.parametrize("name,n,mean", [("c1", 12, None), ("c2", 20, None), ("c2", 16, synth.INTEGRAL),
                                         ("c3", 16, None)])
def test_full_steps_counters_match_oracle(rich, torch, orc, name, n, mean):
    """The FP64 full-step workloads: equal Newton counters, matching records,
    final fields within 1e-8 (fnormtol 1e-12)."""
    r = smooth_recipe(name, n)
    if mean is not None:
        r.problem.mean = mean
    r.options.fnormtol = 1e-12
    r.options.precision = synth.FP64
    out, eg, eo = _run_both(rich, torch, orc, r, 2)
    _compare_counters(out)
    _compare_events(eg, eo, (name, n, mean))
    for sg, so, pg, po in out:
        assert sg["status"] == 0
        assert np.linalg.norm(pg - po) <= 1e-8 * np.linalg.norm(po)


def test_step_phase_stats(rich, torch):
    """The per-phase timers add up and every timed phase moved bytes."""
    r = smooth_recipe("c3", 16)
    s = rich.Solver(r.problem, r.options, torch.from_numpy(r.ks()).to("cuda"))
    s.set_state(torch.from_numpy(r.p0()).to("cuda"))
    st = s.step(2)
    for t in st:
        parts = t["t_feval"] + t["t_jac"] + t["t_aux"] + t["t_setup"] + t["t_linsol"] + t["t_overhead"]
        assert parts == pytest.approx(t["t_total"], rel=1e-9)
        assert t["bytes_feval"] >= 32.0 * r.problem.n * (t["newton_its"] + 1)
        assert t["bytes_linsol"] > 0 and t["bytes_overhead"] > 0
    assert st[0]["t_setup"] > 0 and st[0]["bytes_jac"] > 0
