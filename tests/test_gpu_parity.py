"""HIP library vs the FP64 oracle, element by element, through the C-ABI.

Tolerances (FP64): the two sides evaluate the same formulas with different
pow/exp/log implementations and summation orders, so agreement is at the
level of a few ulps of the largest term; 1e-12 of the row / vector scale is
used.  Integer outputs (patterns, aggregates) must be bit-exact.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from tests.helpers import (all_dirichlet, box_problem, csr_close, random_heads, random_ks,
                           random_spd_graph, smooth_recipe)

pytestmark = pytest.mark.gpu

MEANS = [synth.ARITH, synth.UPSTREAM, synth.HARMONIC, synth.GEOMETRIC, synth.INTEGRAL]


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


def dev(torch, a, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def make_solver(rich, torch, P, ks, opts=None):
    opts = opts or synth.Options()
    return rich.Solver(P, opts, dev(torch, ks))


@pytest.mark.parametrize("mean", MEANS)
@pytest.mark.parametrize("shape", [(13, 11, 9), (1, 1, 40), (64, 3, 5)])
def test_theta_residual(rich, torch, orc, mean, shape):
    P = box_problem(*shape, mean=mean, dt=7.0)
    if shape == (64, 3, 5):
        P.bc_type, P.bc_value = all_dirichlet()
    n = P.n
    ks = random_ks(P, 11)
    p = random_heads(n, 12, saturated_fraction=0.05)
    pold = random_heads(n, 13)
    s = make_solver(rich, torch, P, ks)
    th_g = s.theta(dev(torch, pold)).cpu().numpy()
    th_o = orc.theta(P, pold)
    assert np.max(np.abs(th_g - th_o)) <= 1e-13 * np.max(np.abs(th_o))
    F_g = s.residual(dev(torch, p), dev(torch, th_o)).cpu().numpy()
    F_o = orc.residual(P, ks, p, th_o)
    assert np.max(np.abs(F_g - F_o)) <= 1e-12 * np.max(np.abs(F_o))


@pytest.mark.parametrize("mean", MEANS)
@pytest.mark.parametrize("shape", [(13, 11, 9), (1, 1, 7), (1, 6, 1), (5, 1, 3)])
def test_jacobian_aux_spmv(rich, torch, orc, mean, shape):
    """J and M (CSR and their stencil products) against the oracle; the thin
    shapes have cells with both neighbours absent along a direction."""
    P = box_problem(*shape, mean=mean, dt=3.0)
    n = P.n
    ks = random_ks(P, 21)
    p = random_heads(n, 22, saturated_fraction=0.03)
    s = make_solver(rich, torch, P, ks)
    s.assemble(dev(torch, p))
    rp, col, val = s.export_csr(rich.WHICH_J)
    J = orc.jacobian(P, ks, p)
    csr_close(rp, col, val, J, 1e-12)
    rp, col, val = s.export_csr(rich.WHICH_A, 0)
    M = orc.auxiliary(P, ks, p)
    csr_close(rp, col, val, M, 1e-12)
    x = np.random.default_rng(23).standard_normal(n)
    y = s.apply_jacobian(dev(torch, x)).cpu().numpy()
    yo = J @ x
    assert np.max(np.abs(y - yo)) <= 1e-12 * np.max(np.abs(yo))
    y = s.apply_aux(dev(torch, x)).cpu().numpy()
    yo = M @ x
    assert np.max(np.abs(y - yo)) <= 1e-12 * np.max(np.abs(yo))


@pytest.mark.parametrize("seed", range(6))
def test_match_sweep_bitexact_random(rich, torch, orc, seed):
    n = [1, 2, 17, 300, 1000, 5000][seed]
    A = random_spd_graph(n, min(1.0, 6.0 / max(n, 1)), 100 + seed)
    if seed == 3:  # many exact ties in the weights
        A.data = np.round(A.data * 4) / 4
        A.data[A.data == 0] = -0.25
    agg_o, nc_o = orc.match_sweep(A)
    agg_g, nc_g = rich.match_sweep(dev(torch, A.indptr.astype(np.int64)), dev(torch, A.indices.astype(np.int32)),
                                   dev(torch, A.data.astype(np.float64)))
    assert nc_g == nc_o
    assert np.array_equal(agg_g.cpu().numpy(), agg_o)


def test_match_sweep_empty(rich, torch):
    z64 = torch.zeros(1, dtype=torch.int64, device="cuda")
    agg, nc = rich.match_sweep(z64, torch.zeros(1, dtype=torch.int32, device="cuda"),
                               torch.zeros(1, dtype=torch.float64, device="cuda"))
    assert nc == 0 and agg.numel() == 0


@pytest.mark.parametrize("smoothed", [0, 1, 16])
@pytest.mark.parametrize("mean", MEANS)
def test_hierarchy_bitexact(rich, torch, orc, mean, smoothed):
    """The GPU's set-up on its own M == the oracle's set-up on that same M
    (smoothed: prolongators and coarse matrices equal bit for bit)."""
    P = box_problem(37, 29, 23, mean=mean, dt=10.0)
    n = P.n
    ks = random_ks(P, 31)
    p = random_heads(n, 32, -70, -30)
    opts = synth.Options(amg_coarse_size=200, coarse_dense_max=600, amg_smoothed=smoothed)
    s = make_solver(rich, torch, P, ks, opts)
    s.assemble(dev(torch, p))
    rp, col, val = s.export_csr(rich.WHICH_A, 0)
    M = sp.csr_matrix((val, col, rp), shape=(n, n))
    amg = orc.AMG(opts, M)
    assert s.levels() == amg.levels >= 3
    for l in range(amg.levels):
        Ao, aggo = amg.level(l)
        rp, col, val = s.export_csr(rich.WHICH_A, l)
        csr_close(rp, col, val, Ao, 1e-12)
        if smoothed:
            assert np.array_equal(val, Ao.data)
        if l < amg.levels - 1:
            agg_g, nc = s.export_aggregates(l)
            assert np.array_equal(agg_g, aggo)
            assert np.bincount(agg_g).max() <= 8
            prp, pcol, pval = s.export_csr(rich.WHICH_P, l)
            if l < smoothed:
                Po = amg.prolongator(l)
            else:  # piecewise constant: P(i, agg(i)) = 1
                Po = sp.csr_matrix((np.ones(Ao.shape[0]), (np.arange(Ao.shape[0]), aggo)),
                                   shape=(Ao.shape[0], nc))
            assert np.array_equal(prp, Po.indptr) and np.array_equal(pcol, Po.indices)
            assert np.array_equal(pval, Po.data)
            # the restriction is the prolongator's transpose, columns ascending
            trp, tcol, tval = s.export_csr(rich.WHICH_PT, l)
            PoT = sp.csr_matrix(Po.T)
            PoT.sort_indices()
            assert np.array_equal(trp, PoT.indptr) and np.array_equal(tcol, PoT.indices)
            assert np.array_equal(tval, PoT.data)
    # one V-cycle (FP64) vs the oracle's on the same hierarchy
    b = np.random.default_rng(33).standard_normal(n)
    xg = s.apply_prec(dev(torch, b)).cpu().numpy()
    xo = amg.apply(b)
    assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo)


# gmres_block 1: one Arnoldi vector per Gram-Schmidt round; >= 2: s-step rounds
# (shifted power basis, one block round; 7..10 take the wide-round kernels),
# also where the restart length cuts a round short, on an odd number of rows
# (the kernels' row-pair tail), with every round redone vector by vector
# (gmres_reorth close to 1 rejects each Cholesky factor), with one shift
# instead of the Leja set, at the default tolerance and at one that needs
# restarts.
@pytest.mark.parametrize("block,restart,reorth,n,eta,span", [
    (1, 30, 0.01, 24, 1e-6, 0.55), (5, 30, 0.01, 24, 1e-6, 0.55), (2, 30, 0.01, 23, 1e-6, 0.55),
    (6, 7, 0.01, 23, 1e-6, 0.55), (4, 30, 0.999, 24, 1e-6, 0.55), (5, 30, 0.01, 24, 1e-10, 0.55),
    (3, 10, 0.01, 21, 1e-10, 0.55), (5, 30, 0.01, 24, 1e-6, 0.0), (8, 30, 0.01, 23, 1e-6, 0.55),
    (10, 30, 0.01, 24, 1e-10, 0.55), (9, 30, 0.999, 21, 1e-6, 0.55)])
def test_gmres_parity(rich, torch, orc, block, restart, reorth, n, eta, span):
    r = smooth_recipe("c3", n, precision=synth.FP64)
    r.options.gmres_block, r.options.gmres_restart, r.options.gmres_reorth = block, restart, reorth
    r.options.gmres_shift_span = span
    r.options.eta = eta
    r.options.gmres_maxit = 400
    P = r.problem
    ks, p0 = r.ks(), r.p0()
    s = make_solver(rich, torch, P, ks, r.options)
    th = orc.theta(P, p0)
    F = orc.residual(P, ks, p0, th)
    s.assemble(dev(torch, p0))
    x, its, rr, conv = s.gmres(dev(torch, -F))
    x = x.cpu().numpy()
    rp, col, val = s.export_csr(rich.WHICH_A, 0)
    M = sp.csr_matrix((val, col, rp), shape=(P.n, P.n))
    amg = orc.AMG(r.options, M)
    J = orc.jacobian(P, ks, p0)
    xo, conv_o, its_o, rr_o = orc.gmres(J, -F, amg, r.options.gmres_restart, r.options.eta, r.options.gmres_maxit)
    assert conv and conv_o
    assert abs(its - its_o) <= 1, (its, its_o)
    assert np.linalg.norm(J @ x + F) <= r.options.eta * np.linalg.norm(F) * (1 + 1e-6)
    # both are eta-accurate solutions of the same system: their difference is
    # bounded by the two residuals through ||J^{-1}||; in practice it is far below eta.
    assert np.linalg.norm(x - xo) <= 10 * r.options.eta * np.linalg.norm(xo)


@pytest.mark.parametrize("block,maxit", [(1, 13), (5, 13), (6, 7), (4, 1), (10, 13)])
def test_gmres_iteration_limit(rich, torch, orc, block, maxit):
    """A solve stopped by the iteration limit (mid-round for the s-step
    rounds): the same number of Arnoldi steps as the oracle, neither side
    converged, and the same iterate -- GMRES's k-th iterate is the minimal
    residual point of the same Krylov space whatever the Gram-Schmidt form."""
    r = smooth_recipe("c3", 20, precision=synth.FP64)
    r.options.gmres_block, r.options.gmres_maxit = block, maxit
    r.options.eta = 1e-13  # not reached in maxit steps
    P = r.problem
    ks, p0 = r.ks(), r.p0()
    s = make_solver(rich, torch, P, ks, r.options)
    th = orc.theta(P, p0)
    F = orc.residual(P, ks, p0, th)
    s.assemble(dev(torch, p0))
    x, its, rr, conv = s.gmres(dev(torch, -F))
    x = x.cpu().numpy()
    rp, col, val = s.export_csr(rich.WHICH_A, 0)
    amg = orc.AMG(r.options, sp.csr_matrix((val, col, rp), shape=(P.n, P.n)))
    J = orc.jacobian(P, ks, p0)
    xo, conv_o, its_o, rr_o = orc.gmres(J, -F, amg, r.options.gmres_restart, r.options.eta, maxit)
    assert not conv and not conv_o
    assert its == its_o == maxit
    assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo), np.linalg.norm(x - xo) / np.linalg.norm(xo)


@pytest.mark.parametrize("name,n,mean", [("c1", 12, None), ("c1", 16, None), ("c2", 20, None),
                                         ("c1", 16, synth.GEOMETRIC), ("c2", 16, synth.INTEGRAL)])
def test_full_steps_fp64(rich, torch, orc, name, n, mean):
    r = smooth_recipe(name, n)
    if mean is not None:
        r.problem.mean = mean
    r.options.fnormtol = 1e-12
    r.options.precision = synth.FP64
    P = r.problem
    ks, p = r.ks(), r.p0()
    s = make_solver(rich, torch, P, ks, r.options)
    s.set_state(dev(torch, p))
    o = orc.Solver(P, r.options, ks)
    po = p.copy()
    for step in range(2):
        sg = s.step(1)[0]
        so = o.step(po)
        assert sg["status"] == 0 and so["status"] == 0
        pg = s.get_state().cpu().numpy()
        err = np.linalg.norm(pg - po) / np.linalg.norm(po)
        assert err <= 1e-8, (step, err, sg, so)


@pytest.mark.parametrize("block", [1, 3, 5, 6, 8])
def test_full_steps_gmres_rounds(rich, torch, orc, block):
    """Two FP64 steps of the rough c3 statistics at 16^3 with one-vector
    GMRES rounds and with s-step rounds of 3, 5, 6 and 8 vectors (the
    default of 10 is covered above): the same Newton iterations, Jacobian
    builds and backtracks as the oracle, states within 1e-8."""
    r = smooth_recipe("c3", 16, precision=synth.FP64)
    r.options.fnormtol = 1e-12
    r.options.gmres_block = block
    P = r.problem
    ks, p = r.ks(), r.p0()
    s = make_solver(rich, torch, P, ks, r.options)
    s.set_state(dev(torch, p))
    o = orc.Solver(P, r.options, ks)
    po = p.copy()
    for step in range(2):
        sg = s.step(1)[0]
        so = o.step(po)
        assert sg["status"] == 0 and so["status"] == 0, (step, sg, so)
        for f in ("newton_its", "jac_builds", "ls_backtracks"):
            assert sg[f] == so[f], (step, f, sg[f], so[f])
        pg = s.get_state().cpu().numpy()
        err = np.linalg.norm(pg - po) / np.linalg.norm(po)
        assert err <= 1e-8, (step, err, sg, so)


@pytest.mark.parametrize("smoothed", [0, 1])
def test_full_steps_mixed(rich, torch, orc, smoothed):
    r = smooth_recipe("c3", 24)
    r.options.amg_smoothed = smoothed
    assert r.options.precision == synth.MIXED
    P = r.problem
    ks, p = r.ks(), r.p0()
    s = make_solver(rich, torch, P, ks, r.options)
    s.set_state(dev(torch, p))
    o = orc.Solver(P, r.options, ks)
    po = p.copy()
    for step in range(2):
        sg = s.step(1)[0]
        so = o.step(po)
        assert sg["status"] == 0 and so["status"] == 0
        pg = s.get_state().cpu().numpy()
        err = np.linalg.norm(pg - po) / np.linalg.norm(po)
        assert err <= 1e-6, (step, err, sg, so)


@pytest.mark.parametrize("refresh,smoothed", [(0, 0), (1, 0), (1, 16)])
def test_hierarchy_refresh(rich, torch, orc, refresh, smoothed):
    """After a second assembly the GPU's refreshed hierarchy equals the oracle's
    (aggregates kept; coarse matrices recomputed when refresh = 1)."""
    P = box_problem(33, 27, 21, mean=synth.UPSTREAM, dt=10.0)
    n = P.n
    ks = random_ks(P, 41)
    opts = synth.Options(amg_coarse_size=150, coarse_dense_max=400, amg_refresh=refresh, amg_smoothed=smoothed)
    s = make_solver(rich, torch, P, ks, opts)
    s.assemble(dev(torch, random_heads(n, 42, -70, -30)))
    rp, col, val = s.export_csr(rich.WHICH_A, 0)
    amg = orc.AMG(opts, sp.csr_matrix((val, col, rp), shape=(n, n)))
    s.assemble(dev(torch, random_heads(n, 43, -60, -10)))
    rp, col, val = s.export_csr(rich.WHICH_A, 0)
    amg.update_fine(sp.csr_matrix((val, col, rp), shape=(n, n)))
    assert s.levels() == amg.levels >= 3
    for l in range(amg.levels):
        Ao, aggo = amg.level(l)
        rp, col, val = s.export_csr(rich.WHICH_A, l)
        csr_close(rp, col, val, Ao, 1e-12)
        if l < amg.levels - 1:
            assert np.array_equal(s.export_aggregates(l)[0], aggo)
    b = np.random.default_rng(44).standard_normal(n)
    xg = s.apply_prec(dev(torch, b)).cpu().numpy()
    xo = amg.apply(b)
    assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo)


def test_mixed_vcycle_close_to_fp64(rich, torch, orc):
    """The FP32 V-cycle agrees with the FP64 one to single-precision accuracy."""
    r = smooth_recipe("c3", 20)
    P = r.problem
    ks, p0 = r.ks(), r.p0()
    b = np.random.default_rng(45).standard_normal(P.n)
    out = {}
    for prec in (synth.FP64, synth.MIXED):
        r.options.precision = prec
        s = make_solver(rich, torch, P, ks, r.options)
        s.assemble(dev(torch, p0))
        out[prec] = s.apply_prec(dev(torch, b)).cpu().numpy()
    err = np.linalg.norm(out[synth.MIXED] - out[synth.FP64]) / np.linalg.norm(out[synth.FP64])
    assert err <= 1e-5


def test_aux_dflux_matches_oracle(rich, torch, orc):
    """The optional flux-derivative diagonal of the auxiliary matrix (aux_dflux = 1)."""
    P = box_problem(13, 11, 9, mean=synth.HARMONIC, dt=3.0)
    ks = random_ks(P, 24)
    p = random_heads(P.n, 25, -60, -30)
    opts = synth.Options(aux_dflux=1, amg_max_levels=1, coarse_dense_max=0)
    s = make_solver(rich, torch, P, ks, opts)
    s.assemble(dev(torch, p))
    rp, col, val = s.export_csr(rich.WHICH_A, 0)
    csr_close(rp, col, val, orc.auxiliary(P, ks, p, dflux=True), 1e-12)


@pytest.mark.parametrize("mean,smoothed", [(synth.ARITH, 0), (synth.UPSTREAM, 0), (synth.UPSTREAM, 1)])
def test_vcycle_tiled_stencil(rich, torch, orc, mean, smoothed):
    """Rows of 48+ cells take the tiled fine-level smoother: a ragged grid
    (x: 64 + 36, y: 2 x 8 + 5, z: chunks of 1, 4 (4 x 4 + 3) and 19 planes)
    against the oracle's V-cycle on the same hierarchy (FP64), bit for bit the
    same for every chunk depth, and the FP32 V-cycle against it."""
    P = box_problem(100, 21, 19, mean=mean, dt=10.0)
    n = P.n
    ks = random_ks(P, 51)
    p = random_heads(n, 52, -70, -30)
    b = np.random.default_rng(53).standard_normal(n)
    xs = {}
    for kz in (1, 4, 0):
        opts = synth.Options(precision=synth.FP64, amg_smoothed=smoothed, tile_kz=kz)
        s = make_solver(rich, torch, P, ks, opts)
        s.assemble(dev(torch, p))
        xs[kz] = s.apply_prec(dev(torch, b)).cpu().numpy()
        if kz == 0:
            rp, col, val = s.export_csr(rich.WHICH_A, 0)
            amg = orc.AMG(opts, sp.csr_matrix((val, col, rp), shape=(n, n)))
            assert s.levels() == amg.levels >= 2
        s.close()
    assert np.array_equal(xs[1], xs[4]) and np.array_equal(xs[1], xs[0])
    xo = amg.apply(b)
    assert np.linalg.norm(xs[0] - xo) <= 1e-10 * np.linalg.norm(xo)
    for kz in (4, 0):
        opts = synth.Options(precision=synth.MIXED, amg_smoothed=smoothed, tile_kz=kz)
        s = make_solver(rich, torch, P, ks, opts)
        s.assemble(dev(torch, p))
        xm = s.apply_prec(dev(torch, b)).cpu().numpy()
        s.close()
        assert np.linalg.norm(xm - xo) <= 1e-5 * np.linalg.norm(xo)


@pytest.mark.parametrize("precision,tol", [(synth.FP64, 1e-8), (synth.MIXED, 1e-6)])
def test_paper_3d_case_steps(rich, torch, orc, precision, tol):
    """Section 6's 3-D test (zero-head square on the top face, GMRES(10),
    eta 1e-7) on a reduced 30 x 30 x 6 grid: two steps against the oracle."""
    r = synth.recipe("paper3d", n=30, nz=6, precision=precision)
    if precision == synth.FP64:
        r.options.fnormtol = 1e-12
    P = r.problem
    ks, p = r.ks(), r.p0()
    s = make_solver(rich, torch, P, ks, r.options)
    s.set_state(dev(torch, p))
    th = orc.theta(P, p)
    F_g = s.residual(dev(torch, p), dev(torch, th)).cpu().numpy()
    F_o = orc.residual(P, ks, p, th)
    assert np.max(np.abs(F_g - F_o)) <= 1e-12 * np.max(np.abs(F_o))
    o = orc.Solver(P, r.options, ks)
    po = p.copy()
    for step in range(2):
        sg = s.step(1)[0]
        so = o.step(po)
        assert sg["status"] == 0 and so["status"] == 0
        pg = s.get_state().cpu().numpy()
        err = np.linalg.norm(pg - po) / np.linalg.norm(po)
        assert err <= tol, (step, err, sg, so)


@pytest.mark.parametrize("mean,mean_z", [(synth.ARITH, synth.UPSTREAM), (synth.HARMONIC, synth.INTEGRAL)])
def test_per_direction_means(rich, torch, orc, mean, mean_z):
    """One mean on the x and y faces, another on the z faces: Phi, J and M."""
    P = box_problem(13, 11, 9, mean=mean, dt=3.0)
    P.mean_vertical = mean_z
    ks = random_ks(P, 61)
    p = random_heads(P.n, 62)
    th = orc.theta(P, random_heads(P.n, 63))
    s = make_solver(rich, torch, P, ks)
    F_g = s.residual(dev(torch, p), dev(torch, th)).cpu().numpy()
    F_o = orc.residual(P, ks, p, th)
    assert np.max(np.abs(F_g - F_o)) <= 1e-12 * np.max(np.abs(F_o))
    s.assemble(dev(torch, p))
    rp, col, val = s.export_csr(rich.WHICH_J, 0)
    csr_close(rp, col, val, orc.jacobian(P, ks, p), 1e-12)
    rp, col, val = s.export_csr(rich.WHICH_A, 0)
    csr_close(rp, col, val, orc.auxiliary(P, ks, p), 1e-12)


@pytest.mark.parametrize("smoothed", [0, 1])
def test_vcycle_gauss_seidel(rich, torch, orc, smoothed):
    """The multicolour Gauss-Seidel fine level (smoother = 1) against the
    oracle's V-cycle on the same hierarchy: FP64 to 1e-10, the FP32 V-cycle to
    1e-5, on a ragged grid with three or more levels."""
    P = box_problem(37, 22, 19, mean=synth.UPSTREAM, dt=10.0)
    n = P.n
    ks = random_ks(P, 61)
    p = random_heads(n, 62, -70, -30)
    b = np.random.default_rng(63).standard_normal(n)
    opts = synth.Options(precision=synth.FP64, amg_smoothed=smoothed, smoother=1, amg_coarse_size=150,
                         coarse_dense_max=400)
    s = make_solver(rich, torch, P, ks, opts)
    s.assemble(dev(torch, p))
    xg = s.apply_prec(dev(torch, b)).cpu().numpy()
    rp, col, val = s.export_csr(rich.WHICH_A, 0)
    amg = orc.AMG(opts, sp.csr_matrix((val, col, rp), shape=(n, n)))
    assert s.levels() == amg.levels >= 3
    s.close()
    xo = amg.apply(b)
    assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo)
    # and it is not the l1-Jacobi V-cycle
    opts.smoother = 0
    amg_j = orc.AMG(opts, sp.csr_matrix((val, col, rp), shape=(n, n)))
    assert np.linalg.norm(amg_j.apply(b) - xo) > 1e-3 * np.linalg.norm(xo)
    opts.smoother, opts.precision = 1, synth.MIXED
    s = make_solver(rich, torch, P, ks, opts)
    s.assemble(dev(torch, p))
    xm = s.apply_prec(dev(torch, b)).cpu().numpy()
    s.close()
    assert np.linalg.norm(xm - xo) <= 1e-5 * np.linalg.norm(xo)


@pytest.mark.parametrize("precision,tol", [(synth.FP64, 1e-8), (synth.MIXED, 1e-6)])
def test_full_steps_gauss_seidel(rich, torch, orc, precision, tol):
    r = smooth_recipe("c3", 24)
    r.options.smoother = 1
    r.options.precision = precision
    if precision == synth.FP64:
        r.options.fnormtol = 1e-12
    P = r.problem
    ks, p = r.ks(), r.p0()
    s = make_solver(rich, torch, P, ks, r.options)
    s.set_state(dev(torch, p))
    o = orc.Solver(P, r.options, ks)
    po = p.copy()
    for step in range(2):
        sg = s.step(1)[0]
        so = o.step(po)
        assert sg["status"] == 0 and so["status"] == 0
        pg = s.get_state().cpu().numpy()
        err = np.linalg.norm(pg - po) / np.linalg.norm(po)
        assert err <= tol, (step, err, sg, so)


@pytest.mark.parametrize("block,smoothed", [(4096, 0), (997, 0), (4096, 16)])
@pytest.mark.parametrize("mean", [synth.ARITH, synth.UPSTREAM])
def test_vmb_hierarchy_bitexact(rich, torch, orc, mean, block, smoothed):
    """Decoupled greedy aggregation (amg_aggregation = 1): the GPU's aggregates
    on every level equal the oracle's bit for bit (a ragged last block when the
    block size does not divide the rows), coarse matrices and smoothed
    prolongators as for matching, and one V-cycle agrees."""
    P = box_problem(37, 29, 23, mean=mean, dt=10.0)
    n = P.n
    ks = random_ks(P, 81)
    p = random_heads(n, 82, -70, -30)
    opts = synth.Options(amg_aggregation=1, amg_block=block, amg_smoothed=smoothed, amg_coarse_size=200,
                         coarse_dense_max=600)
    s = make_solver(rich, torch, P, ks, opts)
    s.assemble(dev(torch, p))
    rp, col, val = s.export_csr(rich.WHICH_A, 0)
    amg = orc.AMG(opts, sp.csr_matrix((val, col, rp), shape=(n, n)))
    assert s.levels() == amg.levels >= 3
    for l in range(amg.levels):
        Ao, aggo = amg.level(l)
        rp, col, val = s.export_csr(rich.WHICH_A, l)
        csr_close(rp, col, val, Ao, 1e-12)
        if l < amg.levels - 1:
            agg_g, nc = s.export_aggregates(l)
            assert np.array_equal(agg_g, aggo)
            assert nc == int(aggo.max()) + 1
            if l < smoothed:
                prp, pcol, pval = s.export_csr(rich.WHICH_P, l)
                Po = amg.prolongator(l)
                assert np.array_equal(prp, Po.indptr) and np.array_equal(pcol, Po.indices)
    b = np.random.default_rng(83).standard_normal(n)
    xg = s.apply_prec(dev(torch, b)).cpu().numpy()
    xo = amg.apply(b)
    assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo)


@pytest.mark.parametrize("precision,tol", [(synth.FP64, 1e-8), (synth.MIXED, 1e-6)])
def test_full_steps_vmb(rich, torch, orc, precision, tol):
    r = smooth_recipe("c3", 24)
    r.options.amg_aggregation = 1
    r.options.amg_smoothed = 16
    r.options.precision = precision
    if precision == synth.FP64:
        r.options.fnormtol = 1e-12
    P = r.problem
    ks, p = r.ks(), r.p0()
    s = make_solver(rich, torch, P, ks, r.options)
    s.set_state(dev(torch, p))
    o = orc.Solver(P, r.options, ks)
    po = p.copy()
    for step in range(2):
        sg = s.step(1)[0]
        so = o.step(po)
        assert sg["status"] == 0 and so["status"] == 0
        pg = s.get_state().cpu().numpy()
        err = np.linalg.norm(pg - po) / np.linalg.norm(po)
        assert err <= tol, (step, err, sg, so)


@pytest.mark.parametrize("shape,dense_max", [((1, 1, 1), 4096), ((1, 1, 40), 4096), ((1, 1, 40), 0),
                                             ((3, 2, 1), 4096)])
def test_degenerate_grids_steps(rich, torch, orc, shape, dense_max):
    """A single cell, a vertical column and a flat slab: one-level hierarchies
    (dense direct solve, or l1 sweeps when the dense solve is off) through two
    backward-Euler steps, against the oracle."""
    P = box_problem(*shape, mean=synth.UPSTREAM, dt=5.0)
    opts = synth.Options(precision=synth.FP64, fnormtol=1e-12, coarse_dense_max=dense_max, coarse_l1_sweeps=8,
                         gmres_maxit=400)
    ks = random_ks(P, 91) if P.n > 1 else np.full(1, synth.KS0)
    p = np.full(P.n, synth.P_INIT)
    s = make_solver(rich, torch, P, ks, opts)
    s.set_state(dev(torch, p))
    o = orc.Solver(P, opts, ks)
    po = p.copy()
    for step in range(2):
        sg = s.step(1)[0]
        so = o.step(po)
        assert sg["status"] == 0 and so["status"] == 0, (sg, so)
        pg = s.get_state().cpu().numpy()
        assert np.linalg.norm(pg - po) <= 1e-8 * np.linalg.norm(po), (step, pg[:4], po[:4])
    assert s.levels() == 1


@pytest.mark.parametrize("precision", [synth.FP64, synth.MIXED])
def test_failure_paths_match_oracle(rich, torch, orc, precision):
    """A non-finite head and a Newton iteration limit end the step with the
    oracle's status, and a failed step leaves the previous level in place
    (the error travels back through rich_step's return code and the step's
    statistics)."""
    from paper_2112_05051_amd import _lib
    r = synth.recipe("c1", n=6)
    r.options.precision = precision
    P = r.problem
    ks, p = r.ks(), r.p0()
    bad = p.copy()
    bad[3] = np.nan
    o = orc.Solver(P, r.options, ks)
    assert o.step(bad.copy())["status"] == orc.NONFINITE
    s = make_solver(rich, torch, P, ks, r.options)
    s.set_state(dev(torch, bad))
    with pytest.raises(rich.RichError) as e:
        s.step(1)
    assert e.value.status == _lib.NONFINITE
    s.set_state(dev(torch, bad))
    st = s.step(1, raise_on_error=False)[0]
    assert st["status"] == _lib.NONFINITE
    got = s.get_state().cpu().numpy()
    assert np.array_equal(np.isnan(got), np.isnan(bad)) and np.array_equal(got[~np.isnan(bad)], bad[~np.isnan(bad)])
    s.close()
    # Newton iteration limit at an unreachable tolerance
    r.options.max_newton = 1
    r.options.fnormtol = 1e-30
    o = orc.Solver(P, r.options, ks)
    so = o.step(p.copy())
    s = make_solver(rich, torch, P, ks, r.options)
    s.set_state(dev(torch, p))
    sg = s.step(1, raise_on_error=False)[0]
    assert sg["status"] == so["status"], (sg, so)
    if sg["status"] < 0:
        assert np.array_equal(s.get_state().cpu().numpy(), p)
    s.close()
