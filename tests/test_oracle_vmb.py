"""Pins of the oracle's decoupled greedy aggregation (the DSVMB coarsening of
Section 5.2: Vanek-Mandel-Brezina aggregation applied by each process to its
own rows, here consecutive row blocks).

Independent facts used: hand-worked aggregates of the 1-D Laplacian (one block
and two decoupled blocks) and of the 3 x 3 five-point Laplacian (which goes
through phase 2); on random 3-D auxiliary matrices the invariants of the
construction: a partition into aggregates numbered block by block, no
aggregate across a block boundary, every aggregate connected through strong
couplings, all singletons when nothing is strong; the hierarchy built with it
takes exactly these aggregates and the Galerkin product over them.
"""
from collections import deque

import numpy as np
import scipy.sparse as sp

import synth
from tests.helpers import box_problem, random_heads, random_ks, smooth_recipe


def lap1d(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()


def test_1d_laplacian_one_block(orc):
    agg, nc = orc.vmb_aggregate(lap1d(20), 0.01, 4096)
    assert nc == 7
    assert list(agg) == [0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 3, 4, 4, 4, 5, 5, 5, 6, 6, 6]


def test_1d_laplacian_two_decoupled_blocks(orc):
    agg, nc = orc.vmb_aggregate(lap1d(20), 0.01, 10)
    assert nc == 8
    assert list(agg) == [0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 4, 4, 5, 5, 5, 6, 6, 6, 7, 7]


def test_2d_laplacian_phase_two(orc):
    T = lap1d(3)
    A = (sp.kron(sp.eye(3), T) + sp.kron(T, sp.eye(3))).tocsr()  # c = i + 3 j
    agg, nc = orc.vmb_aggregate(A, 0.01, 4096)
    # roots 0 = {0,1,3} and 5 = {2,4,5,8}; 6 and 7 join their strongest phase-1 neighbours
    assert nc == 2
    assert list(agg) == [0, 0, 1, 0, 1, 1, 0, 1, 1]


def _strong(A, theta):
    d = A.diagonal()
    C = A.tocoo()
    m = (C.row != C.col) & (np.abs(C.data) >= theta * np.sqrt(np.abs(d[C.row] * d[C.col])))
    return sp.csr_matrix((np.ones(m.sum()), (C.row[m], C.col[m])), shape=A.shape)


def test_invariants_random_3d(orc):
    P = box_problem(13, 11, 9)
    A = orc.auxiliary(P, random_ks(P, 71, sigma=2.0), random_heads(P.n, 72, -70, -20)).tocsr()
    for theta, block in ((0.01, 300), (0.25, 4096), (0.5, 257)):
        agg, nc = orc.vmb_aggregate(A, theta, block)
        assert agg.min() >= 0 and set(agg) == set(range(nc))
        blk = np.arange(A.shape[0]) // block
        # numbered block by block, never across a block boundary
        first = {}
        for i, a in enumerate(agg):
            first.setdefault(a, i)
            assert blk[first[a]] == blk[i]
        assert np.all(np.diff([blk[first[a]] for a in range(nc)]) >= 0)
        # connected through strong couplings inside the block
        S = _strong(A, theta)
        members = {}
        for i, a in enumerate(agg):
            members.setdefault(a, []).append(i)
        for a, mem in members.items():
            ms = set(mem)
            seen, q = {mem[0]}, deque([mem[0]])
            while q:
                i = q.popleft()
                for j in S.indices[S.indptr[i]:S.indptr[i + 1]]:
                    if j in ms and j not in seen:
                        seen.add(j)
                        q.append(j)
            assert seen == ms
    agg, nc = orc.vmb_aggregate(A, 10.0, 4096)  # nothing is strong
    assert nc == A.shape[0] and np.array_equal(agg, np.arange(A.shape[0]))


def test_hierarchy_takes_the_aggregates(orc):
    P = box_problem(12, 10, 9)
    A = orc.auxiliary(P, random_ks(P, 73), random_heads(P.n, 74, -70, -30)).tocsr()
    opts = synth.Options(amg_aggregation=1, amg_block=500, amg_coarse_size=20, coarse_dense_max=200)
    amg = orc.AMG(opts, A)
    assert amg.levels >= 3
    for l in range(amg.levels - 1):
        Al, agg = amg.level(l)
        ref, nc = orc.vmb_aggregate(Al, opts.amg_theta, opts.amg_block)
        assert np.array_equal(agg, ref)
        C = orc.galerkin(Al, agg, nc)
        assert abs(amg.level(l + 1)[0] - C).max() <= 1e-12 * abs(C).max()


def test_solver_steps_with_vmb(orc):
    rec = smooth_recipe("c3", 16, precision=synth.FP64)
    rec.options.amg_aggregation = 1
    rec.options.amg_smoothed = 16
    ks, p = rec.ks(), rec.p0().copy()
    S = orc.Solver(rec.problem, rec.options, ks)
    for _ in range(2):
        th_old = orc.theta(rec.problem, p)
        st = S.step(p)
        assert st["status"] == 0, st
        assert np.abs(orc.residual(rec.problem, ks, p, th_old)).max() <= rec.options.fnormtol * (1 + 1e-9)
