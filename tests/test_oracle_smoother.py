"""Pins of the oracle's multicolour Gauss-Seidel smoother (the GPU form of the
hybrid backward/forward Gauss-Seidel smoother the paper's experiments use,
Section 6) and of the V-cycle that applies it on the finest level.

Independent facts used: a greedy colouring in index order of the 7-point grid
graph is the red-black parity (i+j+k) mod 2 (the graph is bipartite and every
lower neighbour of a cell has the other parity); a forward Gauss-Seidel sweep in
the colour-sorted ordering solves (D + L) x_new = b - U x_old and a backward one
(D + U) x_new = b - L x_old, L and U the strict triangles in that ordering
(scipy triangular solves); the V-cycle equals the dense recursion of eq.
(Vcycle) with the backward sweep from zero before and the forward sweep after
the coarse correction on level 0.
"""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import spsolve_triangular

import synth
from tests.helpers import box_problem, random_heads, random_ks, smooth_recipe


def _aux(orc, shape=(7, 6, 5), seed=3):
    P = box_problem(*shape)
    return P, orc.auxiliary(P, random_ks(P, seed), random_heads(P.n, seed + 1, -70, -30)).tocsr()


def test_greedy_colouring_is_red_black(orc):
    P, M = _aux(orc)
    color, nc = orc.greedy_colors(M)
    k, j, i = np.meshgrid(np.arange(P.nz), np.arange(P.ny), np.arange(P.nx), indexing="ij")
    assert nc == 2
    assert np.array_equal(color, ((i + j + k) % 2).ravel())


def _triangles(A, color):
    """Strict lower / upper parts and diagonal of A in the colour-sorted ordering
    (stable: index order within a colour), as matrices in the original indexing."""
    rank = np.empty(A.shape[0], np.int64)
    rank[np.argsort(color, kind="stable")] = np.arange(A.shape[0])
    C = A.tocoo()
    low = rank[C.col] < rank[C.row]
    up = rank[C.col] > rank[C.row]
    L = sp.csr_matrix((C.data[low], (C.row[low], C.col[low])), shape=A.shape)
    U = sp.csr_matrix((C.data[up], (C.row[up], C.col[up])), shape=A.shape)
    return L, sp.diags(A.diagonal()).tocsr(), U, rank


def _solve_in_order(T, rhs, rank, lower):
    """Solve T x = rhs for T triangular in the ordering given by rank."""
    order = np.argsort(rank)
    Tp = T[order][:, order].tocsr()
    xp = spsolve_triangular(Tp, rhs[order], lower=lower)
    x = np.empty_like(xp)
    x[order] = xp
    return x


def test_sweeps_are_triangular_solves(orc):
    _, A = _aux(orc, (6, 5, 4), seed=9)
    color, nc = orc.greedy_colors(A)
    L, D, U, rank = _triangles(A, color)
    rng = np.random.default_rng(10)
    b, x_old = rng.standard_normal(A.shape[0]), rng.standard_normal(A.shape[0])
    fwd = orc.mcgs_sweep(A, color, nc, +1, b, x_old)
    ref = _solve_in_order(D + L, b - U @ x_old, rank, lower=True)
    assert np.linalg.norm(fwd - ref) <= 1e-13 * np.linalg.norm(ref)
    bwd = orc.mcgs_sweep(A, color, nc, -1, b, x_old)
    ref = _solve_in_order(D + U, b - L @ x_old, rank, lower=False)
    assert np.linalg.norm(bwd - ref) <= 1e-13 * np.linalg.norm(ref)
    # a proper colouring makes the sweep independent of the order within a colour:
    # the backward sweep is also the forward sweep of the reversed colour list
    flipped = (nc - 1) - color
    assert np.allclose(orc.mcgs_sweep(A, flipped, nc, +1, b, x_old), bwd, rtol=0, atol=1e-13 * np.abs(bwd).max())


def test_vcycle_with_gauss_seidel_equals_recursion(orc):
    """Dense recursion: level 0 with x0 = (D+U)^-1 b, x1 = x0 + P Mbar_1 P^T (b - A x0),
    x = x1 + (D+L)^-1 (b - A x1); the coarser levels with l1-Jacobi as in Section 5.2."""
    P = box_problem(9, 8, 7)
    M = orc.auxiliary(P, random_ks(P, 6), random_heads(P.n, 7, -70, -30)).tocsr()
    amg = orc.AMG(synth.Options(amg_coarse_size=20, coarse_dense_max=200, smoother=1), M)
    Lv = amg.levels
    assert Lv >= 3 and amg.coarse_dense
    mats, aggs = zip(*[amg.level(l) for l in range(Lv)])
    Mbar = np.linalg.inv(mats[-1].toarray())
    for l in range(Lv - 2, 0, -1):
        Ml = mats[l].toarray()
        n = Ml.shape[0]
        Sinv = np.diag(1.0 / np.abs(Ml).sum(axis=1))
        Pl = np.zeros((n, mats[l + 1].shape[0]))
        Pl[np.arange(n), aggs[l]] = 1.0
        I = np.eye(n)
        Mbar = Sinv.T + Sinv - Sinv.T @ Ml @ Sinv + (I - Sinv.T @ Ml) @ Pl @ Mbar @ Pl.T @ (I - Ml @ Sinv)
    A = mats[0].toarray()
    n = A.shape[0]
    color, _ = orc.greedy_colors(mats[0])
    L, D, U, rank = _triangles(mats[0], color)
    P0 = np.zeros((n, mats[1].shape[0]))
    P0[np.arange(n), aggs[0]] = 1.0
    b = np.random.default_rng(8).standard_normal(n)
    x0 = _solve_in_order(D + U, b, rank, lower=False)
    x1 = x0 + P0 @ (Mbar @ (P0.T @ (b - A @ x0)))
    ref = x1 + _solve_in_order(D + L, b - A @ x1, rank, lower=True)
    x = amg.apply(b)
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)


def test_solver_steps_with_gauss_seidel(orc):
    """Full backward-Euler steps with the Gauss-Seidel fine level reach the Newton
    tolerance (Section 3) like the l1-Jacobi ones."""
    rec = smooth_recipe("c3", 16, precision=synth.FP64)
    rec.options.smoother = 1
    ks, p = rec.ks(), rec.p0().copy()
    S = orc.Solver(rec.problem, rec.options, ks)
    for _ in range(2):
        th_old = orc.theta(rec.problem, p)
        st = S.step(p)
        assert st["status"] == 0, st
        assert np.abs(orc.residual(rec.problem, ks, p, th_old)).max() <= rec.options.fnormtol * (1 + 1e-9)
