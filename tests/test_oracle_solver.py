"""Pins of the oracle's aggregation, V-cycle, GMRES and Newton time stepping.

Matching is checked against the properties that characterise the greedy
matching in a strict edge order (independent code); the Galerkin product
against an explicit P^T A P; the V-cycle against the dense form of the
recursion in Section 5.2; GMRES by finite termination; whole runs by
conservation, the residual tolerance, spectral claims (Section 4) and
symmetry / dimension-reduction invariants.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from tests.helpers import box_problem, random_heads, random_ks, random_spd_graph, smooth_recipe


def edge_key(A, i, j, d):
    lo, hi = min(i, j), max(i, j)
    a = A[lo, hi]
    return (1.0 - (2.0 * a) / (d[lo] + d[hi]), -lo, -hi)  # larger is better


@pytest.mark.parametrize("seed", range(8))
def test_matching_is_the_greedy_matching(orc, seed):
    n = [5, 12, 40, 90, 7, 30, 60, 150][seed]
    A = random_spd_graph(n, 0.3 if n < 50 else 0.08, seed)
    if seed % 2:
        A.data = np.round(A.data * 2) / 2  # exact weight ties -> index tie-breaks
        A.data[A.data == 0] = -0.5
        A.setdiag(np.abs(A.diagonal()) + 1.0)
    A = sp.csr_matrix(A)
    agg, nc = orc.match_sweep(A)
    Ad = A.toarray()
    d = np.diag(Ad)
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if Ad[i, j] != 0]
    groups = {}
    for i, a in enumerate(agg):
        groups.setdefault(a, []).append(i)
    assert sorted(groups) == list(range(nc))
    mate = -np.ones(n, int)
    for a, mem in groups.items():
        assert len(mem) in (1, 2)
        if len(mem) == 2:
            i, j = mem
            assert Ad[min(i, j), max(i, j)] != 0  # a pair is an edge
            mate[i], mate[j] = j, i
    # numbering by smallest member
    mins = [min(groups[a]) for a in range(nc)]
    assert mins == sorted(mins)
    # maximal: no edge joins two singletons
    for i, j in edges:
        assert not (mate[i] < 0 and mate[j] < 0)
    # local dominance certificate: for every matched edge e, an adjacent edge
    # heavier than e must touch a vertex matched by an edge heavier still.
    for i, j in edges:
        if mate[i] != j:
            continue
        ke = edge_key(Ad, i, j, d)
        for v in (i, j):
            for u in range(n):
                if u in (i, j) or (Ad[min(u, v), max(u, v)] == 0):
                    continue
                kf = edge_key(Ad, u, v, d)
                if kf > ke:
                    assert mate[u] >= 0 and edge_key(Ad, u, mate[u], d) > kf


def test_galerkin_equals_explicit_product(orc):
    A = random_spd_graph(200, 0.05, 3)
    agg, nc = orc.match_sweep(A)
    C = orc.galerkin(A, agg, nc)
    P = sp.csr_matrix((np.ones(200), (np.arange(200), agg)), shape=(200, nc))
    ref = (P.T @ A @ P).toarray()
    assert np.allclose(C.toarray(), ref, rtol=1e-14, atol=1e-14 * np.abs(ref).max())
    assert np.all(np.diff(C.indices[C.indptr[0]:C.indptr[1]]) > 0)


def test_hierarchy_shape(orc):
    P = box_problem(20, 18, 17)
    ks = random_ks(P, 4)
    M = orc.auxiliary(P, ks, random_heads(P.n, 5, -70, -30))
    opts = synth.Options(amg_coarse_size=100, coarse_dense_max=400)
    amg = orc.AMG(opts, M)
    assert amg.levels >= 3
    prev = P.n
    for l in range(amg.levels - 1):
        A, agg = amg.level(l)
        counts = np.bincount(agg)
        assert counts.min() >= 1 and counts.max() <= 8  # partition, aggregates of <= 2^3
        nxt, _ = amg.level(l + 1)
        assert nxt.shape[0] == counts.size < prev
        prev = nxt.shape[0]
    assert amg.level(amg.levels - 1)[0].shape[0] <= 100


def test_vcycle_equals_section_5_2_recursion(orc):
    """Dense M-bar_l = S^-T + S^-1 - S^-T M_l S^-1 + (I - S^-T M_l) P M-bar_{l+1} P^T (I - M_l S^-1)
    with S_l the l1 diagonal and M-bar of the coarsest its inverse."""
    P = box_problem(9, 8, 7)
    M = orc.auxiliary(P, random_ks(P, 6), random_heads(P.n, 7, -70, -30))
    opts = synth.Options(amg_coarse_size=20, coarse_dense_max=200)
    amg = orc.AMG(opts, M)
    L = amg.levels
    assert L >= 3 and amg.coarse_dense
    mats, aggs = zip(*[amg.level(l) for l in range(L)])
    Mbar = np.linalg.inv(mats[-1].toarray())
    for l in range(L - 2, -1, -1):
        Ml = mats[l].toarray()
        n = Ml.shape[0]
        Sinv = np.diag(1.0 / np.abs(Ml).sum(axis=1))
        Pl = np.zeros((n, mats[l + 1].shape[0]))
        Pl[np.arange(n), aggs[l]] = 1.0
        I = np.eye(n)
        Mbar = Sinv.T + Sinv - Sinv.T @ Ml @ Sinv + (I - Sinv.T @ Ml) @ Pl @ Mbar @ Pl.T @ (I - Ml @ Sinv)
    b = np.random.default_rng(8).standard_normal(P.n)
    x = amg.apply(b)
    ref = Mbar @ b
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)
    # the V-cycle is symmetric positive definite (a valid preconditioner for CG/GMRES)
    assert np.allclose(Mbar, Mbar.T, atol=1e-12 * np.abs(Mbar).max())
    assert np.linalg.eigvalsh(0.5 * (Mbar + Mbar.T)).min() > 0


@pytest.mark.parametrize("sweeps", [1, 2, 4])
def test_vcycle_with_l1_sweeps_at_the_coarsest(orc, sweeps):
    """When the coarsest level is too large for the direct solve, it takes k
    l1-Jacobi sweeps from zero: M-bar_c = sum_{i<k} (I - D^-1 A_c)^i D^-1 with D the
    l1 diagonal, and the rest of the recursion of Section 5.2 is unchanged."""
    P = box_problem(9, 8, 7)
    M = orc.auxiliary(P, random_ks(P, 6), random_heads(P.n, 7, -70, -30))
    opts = synth.Options(amg_coarse_size=20, coarse_dense_max=0, coarse_l1_sweeps=sweeps)
    amg = orc.AMG(opts, M)
    L = amg.levels
    assert L >= 3 and not amg.coarse_dense
    mats, aggs = zip(*[amg.level(l) for l in range(L)])
    Ac = mats[-1].toarray()
    Dinv = np.diag(1.0 / np.abs(Ac).sum(axis=1))
    E = np.eye(Ac.shape[0]) - Dinv @ Ac
    Mbar = sum(np.linalg.matrix_power(E, i) for i in range(sweeps)) @ Dinv
    for l in range(L - 2, -1, -1):
        Ml = mats[l].toarray()
        n = Ml.shape[0]
        Sinv = np.diag(1.0 / np.abs(Ml).sum(axis=1))
        Pl = np.zeros((n, mats[l + 1].shape[0]))
        Pl[np.arange(n), aggs[l]] = 1.0
        I = np.eye(n)
        Mbar = Sinv.T + Sinv - Sinv.T @ Ml @ Sinv + (I - Sinv.T @ Ml) @ Pl @ Mbar @ Pl.T @ (I - Ml @ Sinv)
    b = np.random.default_rng(8).standard_normal(P.n)
    x = amg.apply(b)
    ref = Mbar @ b
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)
    assert np.allclose(Mbar, Mbar.T, atol=1e-12 * np.abs(Mbar).max())


def test_gmres_finite_termination(orc):
    rng = np.random.default_rng(9)
    n = 25
    A = sp.csr_matrix(np.eye(n) * 4 + rng.standard_normal((n, n)))
    b = rng.standard_normal(n)
    x, conv, its, rr = orc.gmres(A, b, None, restart=n, eta=1e-13, maxit=n)
    assert conv and its <= n
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)
    assert np.allclose(x, np.linalg.solve(A.toarray(), b), rtol=1e-9)


def test_gmres_preconditioned_solves_jacobian(orc):
    P = box_problem(12, 11, 10)
    ks = random_ks(P, 10, sigma=1.0, ell=(4, 4, 2))
    p = np.full(P.n, synth.P_INIT)
    th = orc.theta(P, p)
    F = orc.residual(P, ks, p, th)
    J = orc.jacobian(P, ks, p)
    amg = orc.AMG(synth.Options(amg_coarse_size=50, coarse_dense_max=200), orc.auxiliary(P, ks, p))
    x, conv, its, rr = orc.gmres(J, -F, amg, 30, 1e-10, 200)
    assert conv
    assert np.linalg.norm(J @ x + F) <= 1e-10 * np.linalg.norm(F) * (1 + 1e-9)
    x0, conv0, its0, _ = orc.gmres(J, -F, None, 30, 1e-10, 2000)
    assert its < its0  # the preconditioner helps


# -------------------------------------------------------------- spectra
def _glt_gap(orc, N, mean):
    """1-D: sorted eig(h^2 J) vs sorted samples of the symbol
    kappa(x, t) = (h^2/dt) theta'(p(x)) + K(p(x)) (2 - 2 cos t) (Section 4 theorems)."""
    Lz, dt = 40.0, 0.1
    bc = ((synth.NOFLUX,) * 4 + (synth.DIRICHLET, synth.DIRICHLET), (0,) * 4 + (-61.5, -20.7))
    P = box_problem(1, 1, N - 2, mean=mean, dt=dt, L=(1.0, 1.0, Lz), bc=bc)
    h = P.hz
    z = (np.arange(N - 2) + 1) * h
    prof = lambda zz: -61.5 + 40.8 * 0.5 * (1 + np.tanh((zz - 30.0) / 4.0))
    p = prof(z)
    ks = np.full(N - 2, synth.KS0)
    J = orc.jacobian(P, ks, p).toarray()
    ev = np.sort(np.linalg.eigvals(h * h * J).real)
    m = 1000
    xs = (np.arange(m) + 0.5) / m * Lz
    ts = (np.arange(m) + 0.5) / m * math.pi
    _, s1, K, _ = orc.laws(P, prof(xs), synth.KS0)
    kap = (h * h / dt) * s1[:, None] + K[:, None] * (2 - 2 * np.cos(ts))[None, :]
    q = np.quantile(kap.ravel(), (np.arange(N - 2) + 0.5) / (N - 2))
    gap = np.abs(ev - q) / kap.max()
    return gap.mean()


@pytest.mark.parametrize("mean", [synth.ARITH, synth.UPSTREAM])
def test_glt_symbol_1d(orc, mean):
    gaps = [_glt_gap(orc, N, mean) for N in (50, 100, 200)]
    assert gaps[0] < 8e-3 and gaps[1] < 4e-3 and gaps[2] < 2e-3
    assert gaps[2] < gaps[1] < gaps[0]


def test_preconditioned_spectrum_clusters_at_one(orc):
    """Section 5.2: the diffusion-only operator makes M^{-1} J cluster at 1."""
    r = smooth_recipe("c2", 10)
    P = r.problem
    ks = r.ks()
    p = np.full(P.n, synth.P_INIT)
    J = orc.jacobian(P, ks, p).toarray()
    M = orc.auxiliary(P, ks, p).toarray()
    ev = np.linalg.eigvals(np.linalg.solve(M, J))
    assert np.quantile(np.abs(ev - 1), 0.9) < 0.05
    assert np.all(ev.real > 0.5)


# ------------------------------------------------------------ time steps
def test_step_converges_and_conserves(orc):
    r = synth.recipe("c1", n=10)
    P = r.problem
    ks, p = r.ks(), r.p0()
    S = orc.Solver(P, r.options, ks)
    for _ in range(3):
        pold = p.copy()
        st = S.step(p)
        assert st["status"] == 0
        F = orc.residual(P, ks, p, orc.theta(P, pold))
        assert np.max(np.abs(F)) <= r.options.fnormtol
        assert st["fnorm_inf"] <= r.options.fnormtol
        # water enters through the top only: storage rises
        assert (orc.theta(P, p) - orc.theta(P, pold)).sum() > 0


def test_column_equals_3d(orc):
    """Homogeneous K_s, no-flux sides: every column of a 3-D run equals the 1-D run."""
    r = synth.recipe("c1", n=6)
    r.options.fnormtol = 1e-12
    P = r.problem
    ks = np.full(P.n, synth.KS0)
    p = np.full(P.n, synth.P_INIT)
    S = orc.Solver(P, r.options, ks)
    P1 = synth.Problem(nx=1, ny=1, nz=P.nz, hx=P.hx, hy=P.hy, hz=P.hz, mean=P.mean, dt=P.dt)
    S1 = orc.Solver(P1, r.options, np.full(P.nz, synth.KS0))
    p1 = np.full(P.nz, synth.P_INIT)
    for _ in range(2):
        assert S.step(p)["status"] == 0
        assert S1.step(p1)["status"] == 0
        cols = p.reshape(P.nz, P.ny * P.nx)
        err = np.abs(cols - p1[:, None]).max() / np.abs(p1).max()
        assert err <= 1e-10


def test_xy_symmetry(orc):
    r = synth.recipe("c1", n=7)
    r.options.fnormtol = 1e-12
    P = r.problem
    ks = synth.lognormal_ks((7, 7, 7), synth.KS0, 1.0, (2, 2, 2), 5).reshape(7, 7, 7)
    ks = 0.5 * (ks + ks.transpose(0, 2, 1))  # symmetric under x <-> y
    p = np.full(P.n, synth.P_INIT)
    S = orc.Solver(P, r.options, ks.ravel())
    assert S.step(p)["status"] == 0
    q = p.reshape(7, 7, 7)
    assert np.abs(q - q.transpose(0, 2, 1)).max() <= 1e-9 * np.abs(q).max()


def test_failure_paths(orc):
    r = synth.recipe("c1", n=6)
    P = r.problem
    ks, p = r.ks(), r.p0()
    # non-finite input
    S = orc.Solver(P, r.options, ks)
    bad = p.copy()
    bad[3] = np.nan
    assert S.step(bad)["status"] == orc.NONFINITE
    # Newton iteration limit
    r.options.max_newton = 1
    r.options.fnormtol = 1e-30
    S = orc.Solver(P, r.options, ks)
    q = p.copy()
    st = S.step(q)
    assert st["status"] in (orc.MAXITER, orc.STEP_TOO_SMALL, orc.LINESEARCH_FAIL)
    assert np.array_equal(q, p) or st["status"] == orc.STEP_TOO_SMALL


def test_paper_3d_case_patch_and_symmetry(orc):
    """Section 6's 3-D test: a zero-head square on the top face.  Phi changes
    only in the top-layer cells under the square (counted independently from
    the node coordinates), and the solution keeps the square's symmetries
    (x <-> y and both mirrors) after two steps."""
    r = synth.recipe("paper3d", n=20, nz=5)
    r.options.precision = synth.FP64
    P = r.problem
    ks, p = r.ks(), r.p0()
    th = orc.theta(P, p)
    F1 = orc.residual(P, ks, p, th)
    P0 = synth.recipe("paper3d", n=20, nz=5).problem
    P0.patch_face = -1
    F0 = orc.residual(P0, ks, p, th)
    changed = np.abs(F1 - F0).reshape(P.nz, P.ny, P.nx) > 0
    x = (np.arange(P.nx) + 1) * P.hx
    y = (np.arange(P.ny) + 1) * P.hy
    inside = ((x >= 16) & (x <= 48))[None, :] & ((y >= 16) & (y <= 48))[:, None]
    assert inside.sum() > 0 and np.array_equal(changed[-1], inside) and not changed[:-1].any()
    S = orc.Solver(P, r.options, ks)
    for _ in range(2):
        st = S.step(p)
        assert st["status"] == 0
    p3 = p.reshape(P.nz, P.ny, P.nx)
    scale = np.abs(p3).max()
    for q in (p3.transpose(0, 2, 1), p3[:, :, ::-1], p3[:, ::-1, :]):
        assert np.abs(p3 - q).max() <= 1e-10 * scale
    assert p3[-1][inside].max() > P.bc_value[0] + 1.0  # water entered under the square
