"""Pins of the oracle's smoothed aggregation (Section 5.2: the paper's SMATCH and
DSVMB coarsening both smooth the piecewise-constant prolongator).

Independent facts used: in 1-D, damped-Jacobi smoothing (omega = 2/3 for the
Laplacian) of the aggregates {3J, 3J+1, 3J+2} yields the linear-interpolation
hat functions of a grid three times coarser, and the Galerkin operator is then
1/3 of the coarse Laplacian; a Jacobi step with omega below 2/rho(D^-1 A) lowers
the A-energy of every coarse basis function; the pattern of P is the set of
aggregates a row's neighbourhood touches (brute force); P^T A P is the matrix of
the bilinear form (P x)^T A (P y); the V-cycle with smoothed P equals the dense
recursion of eq. (Vcycle).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from tests.helpers import box_problem, random_heads, random_ks, smooth_recipe


def laplacian_1d(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()


def test_1d_hat_functions_and_coarse_laplacian(orc):
    m = 12
    n = 3 * m
    A = laplacian_1d(n)
    agg = np.repeat(np.arange(m), 3).astype(np.int32)
    P, omega = orc.smoothed_prolongator(A, agg, m)
    assert omega == pytest.approx(2.0 / 3.0, rel=1e-15)
    Pd = P.toarray()
    hat = np.array([1 / 3, 2 / 3, 1.0, 2 / 3, 1 / 3])
    for J in range(1, m - 1):
        col = Pd[:, J]
        assert np.allclose(col[3 * J - 1:3 * J + 4], hat, rtol=0, atol=1e-15)
        assert np.all(col[:3 * J - 1] == 0) and np.all(col[3 * J + 4:] == 0)
    C = orc.rap(A, P).toarray()
    for J in range(2, m - 2):
        assert C[J, J] == pytest.approx(2 / 3, rel=1e-14)
        assert C[J, J - 1] == pytest.approx(-1 / 3, rel=1e-14)
        assert C[J, J + 1] == pytest.approx(-1 / 3, rel=1e-14)
        assert np.all(np.abs(np.delete(C[J], [J - 1, J, J + 1])) <= 1e-15)


def _aux_and_aggregates(orc, shape=(9, 8, 7), seed=6):
    P = box_problem(*shape)
    M = orc.auxiliary(P, random_ks(P, seed), random_heads(P.n, seed + 1, -70, -30)).tocsr()
    amg = orc.AMG(synth.Options(amg_coarse_size=20, coarse_dense_max=200), M)
    _, agg = amg.level(0)
    return M, agg, int(agg.max()) + 1


def test_pattern_is_touched_aggregates(orc):
    M, agg, nc = _aux_and_aggregates(orc)
    P, _ = orc.smoothed_prolongator(M, agg, nc)
    for i in range(M.shape[0]):
        touched = sorted({int(agg[k]) for k in M.indices[M.indptr[i]:M.indptr[i + 1]]})
        assert list(P.indices[P.indptr[i]:P.indptr[i + 1]]) == touched


def test_smoothing_lowers_energy_and_omega_is_safe(orc):
    M, agg, nc = _aux_and_aggregates(orc)
    P, omega = orc.smoothed_prolongator(M, agg, nc)
    n = M.shape[0]
    Pt = sp.csr_matrix((np.ones(n), (np.arange(n), agg)), shape=(n, nc))
    D = M.diagonal()
    lam = np.linalg.eigvals(np.diag(1 / D) @ M.toarray()).real.max()
    assert 0 < omega <= 4.0 / (3.0 * lam) * (1 + 1e-12)
    e_s = np.asarray((P.multiply(M @ P)).sum(axis=0)).ravel()      # p_J^T A p_J
    e_t = np.asarray((Pt.multiply(M @ Pt)).sum(axis=0)).ravel()
    assert np.all(e_s < e_t)
    # columns still sum to the same aggregate weight where A has zero row sums:
    # P 1 = (I - omega D^-1 A) 1, checked row by row
    one = np.ones(nc)
    assert np.allclose(P @ one, 1 - omega * (M @ np.ones(n)) / D, rtol=0, atol=1e-13)


def test_rap_is_the_bilinear_form(orc):
    M, agg, nc = _aux_and_aggregates(orc)
    P, _ = orc.smoothed_prolongator(M, agg, nc)
    C = orc.rap(M, P)
    rng = np.random.default_rng(3)
    for _ in range(3):
        x, y = rng.standard_normal(nc), rng.standard_normal(nc)
        lhs = x @ (C @ y)
        rhs = (P @ x) @ (M @ (P @ y))
        assert lhs == pytest.approx(rhs, rel=1e-12)
    Cd = C.toarray()
    assert np.allclose(Cd, Cd.T, rtol=0, atol=1e-14 * np.abs(Cd).max())
    assert np.linalg.eigvalsh(Cd).min() > 0


@pytest.mark.parametrize("smoothed", [1, 16])
def test_smoothed_vcycle_equals_section_5_2_recursion(orc, smoothed):
    """smoothed = 1: only the finest prolongator is smoothed; 16: all of them."""
    P = box_problem(9, 8, 7)
    M = orc.auxiliary(P, random_ks(P, 6), random_heads(P.n, 7, -70, -30))
    opts = synth.Options(amg_coarse_size=20, coarse_dense_max=200, amg_smoothed=smoothed)
    amg = orc.AMG(opts, M)
    L = amg.levels
    assert L >= 3 and amg.coarse_dense
    mats = [amg.level(l)[0] for l in range(L)]
    Mbar = np.linalg.inv(mats[-1].toarray())
    for l in range(L - 2, -1, -1):
        Ml = mats[l].toarray()
        n = Ml.shape[0]
        Sinv = np.diag(1.0 / np.abs(Ml).sum(axis=1))
        Ps = amg.prolongator(l)
        assert (Ps is not None) == (l < smoothed)
        if Ps is None:
            Pl = np.zeros((n, mats[l + 1].shape[0]))
            Pl[np.arange(n), amg.level(l)[1]] = 1.0
        else:
            Pl = Ps.toarray()
        assert Pl.shape == (n, mats[l + 1].shape[0])
        I = np.eye(n)
        Mbar = Sinv.T + Sinv - Sinv.T @ Ml @ Sinv + (I - Sinv.T @ Ml) @ Pl @ Mbar @ Pl.T @ (I - Ml @ Sinv)
        # every stored coarse matrix is the Galerkin product of its fine level
        Cl = mats[l + 1].toarray()
        assert np.allclose(Cl, Pl.T @ Ml @ Pl, rtol=0, atol=1e-13 * np.abs(Cl).max())
    b = np.random.default_rng(8).standard_normal(P.n)
    x = amg.apply(b)
    ref = Mbar @ b
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)


def test_refresh_recomputes_prolongator_and_product(orc):
    P = box_problem(10, 9, 8)
    ks = random_ks(P, 11)
    M1 = orc.auxiliary(P, ks, random_heads(P.n, 12, -70, -30)).tocsr()
    M2 = orc.auxiliary(P, ks, random_heads(P.n, 13, -60, -10)).tocsr()
    opts = synth.Options(amg_coarse_size=20, coarse_dense_max=200, amg_smoothed=16)
    amg = orc.AMG(opts, M1)
    amg.update_fine(M2)
    _, agg = amg.level(0)
    nc = amg.level(1)[0].shape[0]
    P2, _ = orc.smoothed_prolongator(M2, agg, nc)
    assert (amg.prolongator(0) != P2).nnz == 0
    C = amg.level(1)[0]
    assert (C != orc.rap(M2, P2)).nnz == 0


def test_smoothing_reduces_gmres_iterations(orc):
    r = smooth_recipe("c3", 20, precision=synth.FP64)
    P = r.problem
    ks, p = r.ks(), r.p0()
    th = orc.theta(P, p)
    F = orc.residual(P, ks, p, th - 1e-3 * np.abs(th))
    J = orc.jacobian(P, ks, p)
    M = orc.auxiliary(P, ks, p)
    its = {}
    for sm in (0, 1, 16):
        r.options.amg_smoothed = sm
        amg = orc.AMG(r.options, M)
        x, conv, its[sm], _ = orc.gmres(J, -F, amg, 30, 1e-8, 300)
        assert conv
    assert its[1] < its[0] and its[16] < its[0]
