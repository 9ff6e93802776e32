"""The harmonic interface mean (named in the paper's abstract) on the GPU
against the oracle.

A 12^3 block at the 512^3 cube's spacing with that recipe's lognormal K_s
statistics converges at dt = 3 s (the uniform top-layer mode of the Jacobian
is positive there; at the recipe's 30 s it is not and Newton cannot converge,
as the CPU tests in tests/test_oracle_harmonic.py show).  FP64 steps must
match the oracle's to 1e-8 with equal Newton counters, mixed steps to 1e-6.

A run that diverges (a rough harmonic request whose Newton iterates run off
to heads of -1e9 cm) must end with the oracle's status: the FP32 copies of
the preconditioner saturate instead of overflowing, so the mixed path keeps
finite numbers and reaches the same Newton iteration limit.  That holds for
GMRES with one Arnoldi vector per round, whose failing solves follow the
oracle's; the s-step rounds return other (equally unconverged) corrections
from the failing solves, so their Newton path may differ: such a run either
fails the same way or ends at a state the oracle confirms as a root.
"""
import dataclasses

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

H_C5 = 64.0 / 513.0


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


@pytest.mark.parametrize("precision", [synth.FP64, synth.MIXED])
def test_harmonic_block_steps_match_oracle(rich, torch, orc, precision):
    r = synth.recipe("c5", n=12)
    P, ks, p0 = r.problem, r.ks(), r.p0()
    P.hx = P.hy = P.hz = H_C5
    P.dt = 3.0
    r.options.precision = precision
    if precision == synth.FP64:
        r.options.fnormtol = 1e-12
    s = rich.Solver(P, r.options, torch.from_numpy(ks).cuda())
    s.set_state(torch.from_numpy(p0).cuda())
    o = orc.Solver(P, r.options, ks)
    po = p0.copy()
    for step in range(3):
        sg = s.step(1)[0]
        so = o.step(po)
        assert sg["status"] == 0 and so["status"] == 0, (step, sg, so)
        pg = s.get_state().cpu().numpy()
        err = np.linalg.norm(pg - po) / np.linalg.norm(po)
        if precision == synth.FP64:
            assert err <= 1e-8, (step, err)
            for f in ("newton_its", "jac_builds", "ls_backtracks"):
                assert sg[f] == so[f], (step, f, sg[f], so[f])
        else:
            assert err <= 1e-6, (step, err)


def test_diverging_harmonic_request_ends_with_the_oracles_status(rich, torch, orc):
    _, r = synth.serving_stream(count=40, sizes=(32,), nsteps=1)[2]
    assert r.problem.mean == synth.HARMONIC
    r.options.gmres_maxit = 30
    r.options.max_newton = 260
    P, ks, p0 = r.problem, r.ks(), r.p0()
    r.options.precision = synth.FP64
    o = orc.Solver(P, r.options, ks)
    po = p0.copy()
    so = o.step(po)
    assert so["status"] == orc.MAXITER
    assert o.iterate(P.n).min() < -1e9  # the oracle's iterate ran off
    r.options.precision = synth.MIXED
    assert r.options.gmres_block > 1
    for block in (1, r.options.gmres_block):
        o1 = dataclasses.replace(r.options, gmres_block=block)
        s = rich.Solver(P, o1, torch.from_numpy(ks).cuda())
        s.set_state(torch.from_numpy(p0).cuda())
        sg = s.step(1, raise_on_error=False)[0]
        pg = s.get_state().cpu().numpy()
        s.close()
        if block == 1 or sg["status"] != 0:
            assert sg["status"] == so["status"], (block, sg, so)
            assert np.array_equal(pg, p0)  # a failed step leaves the previous level
        else:
            F = orc.residual(P, ks, pg, orc.theta(P, p0))
            assert np.isfinite(pg).all() and np.max(np.abs(F)) <= r.options.fnormtol, (block, np.max(np.abs(F)))
