"""Ensemble server: every request's result in the mix equals its result alone,
with the preconditioned products of the resident simulations fused into
batched launches (plain or persistent) and without; served results against
the oracle."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def small_requests(count=6, steps=3, seed=7, sizes=(10, 12, 14, 16, 18)):
    out = [rec for t, rec in synth.serving_stream(count=count, seed=seed, sizes=sizes, nsteps=steps)]
    for rec in out:
        rec.options.max_newton = 40  # bounds the cost of a request that does not converge
    return out


def run_alone(rich, torch, rec):
    s = rich.Solver(rec.problem, rec.options, torch.from_numpy(rec.ks()).cuda())
    s.set_state(torch.from_numpy(rec.p0()).cuda())
    stats = s.step(rec.nsteps, raise_on_error=False)
    return s.get_state().cpu().numpy(), stats


def check_alone_equals_mix(rich, torch, srv, reqs, ids):
    for rec, i in zip(reqs, ids):
        r = srv.poll(i)
        assert r is not None
        p_alone, st_alone = run_alone(rich, torch, rec)
        # same statuses, same iteration history, same final state bit for bit
        assert [s["status"] for s in r["stats"]] == [s["status"] for s in st_alone[:len(r["stats"])]]
        assert np.array_equal(r["p"], p_alone), np.abs(r["p"] - p_alone).max()
        assert [s["newton_its"] for s in r["stats"]] == [s["newton_its"] for s in st_alone[:len(r["stats"])]]
        assert [s["gmres_its"] for s in r["stats"]] == [s["gmres_its"] for s in st_alone[:len(r["stats"])]]


@pytest.mark.parametrize("fused,persistent", [(True, False), (True, True), (False, False)])
def test_alone_equals_mix(fused, persistent):
    import torch

    import paper_2112_05051_amd as rich
    reqs = small_requests()
    srv = rich.Server(8 << 30, 3, fused=fused, persistent=persistent)
    ids = [srv.submit(rec.problem, rec.options, rec.ks(), rec.p0(), rec.nsteps) for rec in reqs]
    srv.run_until_idle()
    check_alone_equals_mix(rich, torch, srv, reqs, ids)
    flushes, products = srv.batch_stats()
    if fused:
        assert flushes > 0 and products >= flushes  # the products went through the batchers
    else:
        assert flushes == 0 and products == 0
    srv.close()


@pytest.mark.parametrize("persistent", [False, True])
def test_fused_kernels_all_paths(persistent):
    """48^3 grids run the tiled fine smoother and have a CSR-stream coarse
    level, 16^3 grids the plain fine kernels; simulations of one size share
    batched launches (plain, or persistent grids taking their blocks from a
    device work queue), and every result equals the lone run bit for bit."""
    import torch

    import paper_2112_05051_amd as rich
    reqs = []
    for seed, n in ((11, 48), (12, 48), (13, 16), (14, 16)):
        rec = synth.serving_stream(count=1, seed=seed, sizes=(n,), nsteps=2)[0][1]
        rec.problem.mean = synth.UPSTREAM  # converges on these fields
        rec.options.max_newton = 40
        reqs.append(rec)
    srv = rich.Server(16 << 30, 4, fused=True, persistent=persistent)
    ids = [srv.submit(rec.problem, rec.options, rec.ks(), rec.p0(), rec.nsteps) for rec in reqs]
    srv.run_until_idle()
    flushes, products = srv.batch_stats()
    assert flushes > 0 and products > flushes, (flushes, products)
    check_alone_equals_mix(rich, torch, srv, reqs, ids)
    # the tiled-size simulations ran Newton steps (and so fused GMRES products)
    for i in ids[:2]:
        assert sum(s["gmres_its"] for s in srv.poll(i)["stats"]) > 0
    srv.close()


@pytest.mark.parametrize("persistent", [False, True])
def test_fused_fp64(persistent):
    """The all-FP64 batched V-cycle: two same-size FP64 simulations share
    batches and each equals its lone run bit for bit."""
    import torch

    import paper_2112_05051_amd as rich
    reqs = []
    for seed in (21, 22):
        rec = synth.serving_stream(count=1, seed=seed, sizes=(24,), nsteps=2)[0][1]
        rec.problem.mean = synth.ARITH
        rec.options.precision = synth.FP64
        rec.options.max_newton = 40
        reqs.append(rec)
    srv = rich.Server(8 << 30, 2, fused=True, persistent=persistent)
    ids = [srv.submit(rec.problem, rec.options, rec.ks(), rec.p0(), rec.nsteps) for rec in reqs]
    srv.run_until_idle()
    flushes, products = srv.batch_stats()
    assert flushes > 0 and products > flushes, (flushes, products)
    check_alone_equals_mix(rich, torch, srv, reqs, ids)
    srv.close()


def test_fused_mixed_hierarchies():
    """Same-size simulations whose hierarchies differ share a batcher: a
    smoothed-prolongator one (not batchable: it launches on its own stream), a
    greedy-aggregation one (large aggregates: the restriction's unstaged path)
    and plain ones; every result equals its lone run bit for bit."""
    import torch

    import paper_2112_05051_amd as rich
    reqs = []
    for seed, tweak in ((31, {}), (32, {"amg_smoothed": 1}), (33, {"amg_aggregation": 1}), (34, {})):
        rec = synth.serving_stream(count=1, seed=seed, sizes=(20,), nsteps=2)[0][1]
        rec.problem.mean = synth.UPSTREAM
        rec.options.max_newton = 40
        for k, v in tweak.items():
            setattr(rec.options, k, v)
        reqs.append(rec)
    srv = rich.Server(8 << 30, 4, fused=True)
    ids = [srv.submit(rec.problem, rec.options, rec.ks(), rec.p0(), rec.nsteps) for rec in reqs]
    srv.run_until_idle()
    flushes, products = srv.batch_stats()
    assert flushes > 0
    check_alone_equals_mix(rich, torch, srv, reqs, ids)
    srv.close()


def test_budget_serialises_but_completes():
    import paper_2112_05051_amd as rich
    reqs = small_requests(count=4, steps=2, seed=8, sizes=(14,))
    need = max(rich.query_bytes(rec.problem, rec.options) + 16 * rec.problem.n for rec in reqs)
    srv = rich.Server(need + 1024, 4)  # room for one simulation at a time
    ids = [srv.submit(rec.problem, rec.options, rec.ks(), rec.p0(), rec.nsteps) for rec in reqs]
    srv.run_until_idle()
    res = [srv.poll(i) for i in ids]
    assert all(r is not None and r["status"] == 0 for r in res)
    # one at a time: total resident time is the sum of the parts, so the last
    # request waited at least as long as all earlier ones ran
    assert res[-1]["wait_s"] >= 0.9 * sum(r["run_s"] for r in res[:-1])
    srv.close()


def test_served_results_match_the_oracle(orc):
    """FP64 requests of several sizes and interface means served together:
    each served result equals the oracle's run of the same request (rel. L2
    <= 1e-8 at fnormtol 1e-12) with the same Newton counters; a request the
    oracle cannot converge fails on the server too.  The server is created on
    a caller's stream and its requests are ordered after it."""
    import torch

    import paper_2112_05051_amd as rich
    reqs = small_requests(count=8, steps=2, seed=4, sizes=(10, 12, 14, 16, 18))
    for rec in reqs:
        rec.options.precision = synth.FP64
        rec.options.fnormtol = 1e-12
        rec.options.max_newton = 30
    stream = torch.cuda.Stream()
    srv = rich.Server(8 << 30, 4, stream=stream)
    ids = [srv.submit(rec.problem, rec.options, rec.ks(), rec.p0(), rec.nsteps) for rec in reqs]
    srv.run_until_idle()
    converged = 0
    for rec, i in zip(reqs, ids):
        r = srv.poll(i)
        o = orc.Solver(rec.problem, rec.options, rec.ks())
        po = rec.p0().copy()
        so = []
        for _ in range(rec.nsteps):
            so.append(o.step(po))
            if so[-1]["status"] < 0:
                break
        if so[-1]["status"] < 0:
            assert r["status"] < 0, (rec.name, r["status"], so[-1]["status"])
            continue
        converged += 1
        assert r["status"] == 0, (rec.name, r["status"])
        err = np.linalg.norm(r["p"] - po) / np.linalg.norm(po)
        assert err <= 1e-8, (rec.name, err)
        for sg, s_o in zip(r["stats"], so):
            for f in ("newton_its", "jac_builds", "ls_backtracks"):
                assert sg[f] == s_o[f], (rec.name, f, sg[f], s_o[f])
    assert converged >= 5
    srv.close()
