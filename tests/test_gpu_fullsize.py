"""The benchmark-size workloads on the GPU, through the C-ABI, in the launch
configuration the benchmark uses (the recipes' own grids and options): the
128^3 and 256^3 cubes and the paper's 3-D test at its full 798 x 798 x 38.

At these sizes the oracle cannot run the solver in seconds, so the tests check
what it can compute directly: theta and Phi element by element on the full
fields, the oracle's own residual at the GPU's solution (every accepted time
step must satisfy the Newton tolerance of Section 3 whatever path led to it),
and, at 128^3, the level-0 aggregates and level-1 matrix of the GPU's AMG set-up
against the oracle's set-up on the same auxiliary matrix.
"""
import dataclasses

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from tests.helpers import csr_close

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_full_size_step(rich, torch, orc, name):
    rec = synth.recipe(name)
    P = rec.problem
    assert P.n in (128 ** 3, 256 ** 3)
    ks, p0 = rec.ks(), rec.p0()
    s = rich.Solver(P, rec.options, torch.from_numpy(ks).cuda())
    p0_d = torch.from_numpy(p0).cuda()
    # theta and Phi on the full initial field
    th_o = orc.theta(P, p0)
    th_g = s.theta(p0_d).cpu().numpy()
    assert np.max(np.abs(th_g - th_o)) <= 1e-13 * np.max(np.abs(th_o))
    rng = np.random.default_rng(7)
    p1 = p0 + rng.uniform(0.0, 30.0, P.n)           # a perturbed state with active fronts
    F_o = orc.residual(P, ks, p1, th_o)
    F_g = s.residual(torch.from_numpy(p1).cuda(), torch.from_numpy(th_o).cuda()).cpu().numpy()
    assert np.max(np.abs(F_g - F_o)) <= 1e-12 * np.max(np.abs(F_o))
    # one backward-Euler step; the oracle's residual at the GPU's state meets the tolerance
    s.set_state(p0_d)
    st = s.step(1)[0]
    assert st["status"] == 0, st
    pg = s.get_state().cpu().numpy()
    F = orc.residual(P, ks, pg, th_o)
    assert np.max(np.abs(F)) <= rec.options.fnormtol * (1 + 1e-6), (np.max(np.abs(F)), st)
    assert np.all(np.isfinite(pg))
    s.close()


def test_full_size_hierarchy_c2(rich, torch, orc):
    """128^3: the GPU's level-0 matching and level-1 Galerkin matrix equal the
    oracle's on the GPU's own auxiliary matrix."""
    rec = synth.recipe("c2")
    P = rec.problem
    ks, p0 = rec.ks(), rec.p0()
    s = rich.Solver(P, rec.options, torch.from_numpy(ks).cuda())
    s.assemble(torch.from_numpy(p0).cuda())
    rp, col, val = s.export_csr(rich.WHICH_A, 0)
    M = sp.csr_matrix((val, col, rp), shape=(P.n, P.n))
    csr_close(rp, col, val, orc.auxiliary(P, ks, p0), 1e-12)
    # the composed aggregates of the pairwise matching sweeps (Section 5.2)
    agg_o, B = np.arange(P.n), M
    for _ in range(rec.options.amg_sweeps):
        a, nc = orc.match_sweep(B)
        if nc == B.shape[0]:
            break
        agg_o = a[agg_o]
        B = orc.galerkin(B, a, nc)
    nc_o = B.shape[0]
    agg_g, nc_g = s.export_aggregates(0)
    assert nc_g == nc_o and np.array_equal(agg_g, agg_o)
    A1 = orc.galerkin(M, agg_o.astype(np.int32), nc_o)
    rp1, col1, val1 = s.export_csr(rich.WHICH_A, 1)
    csr_close(rp1, col1, val1, A1, 1e-12)
    s.close()


def test_paper_3d_full_size_step(rich, torch, orc):
    """The paper's 3-D infiltration test at its real size (24.2 M unknowns,
    the zero-head patch on the top face): theta and Phi on the full fields, and
    the oracle's residual at the GPU's state after the first step."""
    rec = synth.recipe("paper3d")
    P = rec.problem
    assert (P.nx, P.ny, P.nz) == (798, 798, 38)
    ks, p0 = rec.ks(), rec.p0()
    s = rich.Solver(P, rec.options, torch.from_numpy(ks).cuda())
    p0_d = torch.from_numpy(p0).cuda()
    th_o = orc.theta(P, p0)
    assert np.max(np.abs(s.theta(p0_d).cpu().numpy() - th_o)) <= 1e-13 * np.max(np.abs(th_o))
    s.set_state(p0_d)
    st = s.step(1)[0]
    assert st["status"] == 0, st
    pg = s.get_state().cpu().numpy()
    F = orc.residual(P, ks, pg, th_o)
    assert np.max(np.abs(F)) <= rec.options.fnormtol * (1 + 1e-6), (np.max(np.abs(F)), st)
    # the patch is wetting the top layer: heads there rose from h_r
    top = pg.reshape(P.nz, P.ny, P.nx)[-1]
    assert top.max() > p0.max() + 1.0
    s.close()


def test_full_size_vcycle_and_gmres_c2(rich, torch, orc):
    """128^3 (2^21 rows: the wide Gram-Schmidt kernels of large grids): one
    FP64 V-cycle on the GPU's own auxiliary matrix equals the oracle's V-cycle
    on that matrix (Section 5.2), and one GMRES(30) solve of a Newton
    correction, with s-step rounds and with the speculative one-vector
    Arnoldi steps, matches the oracle's (iterations within one, solutions
    within 10 eta; Section 6's stopping rule)."""
    rec = synth.recipe("c2")
    P, opts = rec.problem, rec.options
    assert P.n == 1 << 21 and opts.precision == synth.FP64
    ks, p0 = rec.ks(), rec.p0()
    rng = np.random.default_rng(7)
    p1 = p0.copy()
    p1.reshape(P.nz, P.ny, P.nx)[-8:] += rng.uniform(0.0, 35.0, (8, P.ny, P.nx))  # a wetted top band
    th = orc.theta(P, p0)
    F = orc.residual(P, ks, p1, th)
    s = rich.Solver(P, opts, torch.from_numpy(ks).cuda())
    s.assemble(torch.from_numpy(p1).cuda())
    rp, col, val = s.export_csr(rich.WHICH_A, 0)
    amg = orc.AMG(opts, sp.csr_matrix((val, col, rp), shape=(P.n, P.n)))
    assert s.levels() == amg.levels >= 3
    b = -F
    xg = s.apply_prec(torch.from_numpy(b).cuda()).cpu().numpy()
    xo = amg.apply(b)
    assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo)
    J = orc.jacobian(P, ks, p1)
    xo, conv_o, its_o, rr_o = orc.gmres(J, b, amg, opts.gmres_restart, opts.eta, opts.gmres_maxit)
    assert conv_o and its_o > opts.gmres_restart  # at least one restart
    # the s-step rounds of the default options, then one Arnoldi vector per round
    assert opts.gmres_block > 1
    for block in (opts.gmres_block, 1):
        if block != opts.gmres_block:
            s.close()
            o1 = dataclasses.replace(opts, gmres_block=block)
            s = rich.Solver(P, o1, torch.from_numpy(ks).cuda())
            s.assemble(torch.from_numpy(p1).cuda())
        x, its, rr, conv = s.gmres(torch.from_numpy(b).cuda())
        x = x.cpu().numpy()
        assert conv
        assert abs(its - its_o) <= 1, (block, its, its_o)
        assert np.linalg.norm(J @ x - b) <= opts.eta * np.linalg.norm(b) * (1 + 1e-6)
        assert np.linalg.norm(x - xo) <= 10 * opts.eta * np.linalg.norm(xo)
    s.close()
