"""Shared input builders for the tests (seeded, synthetic; no method arithmetic)."""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

import synth


def box_problem(nx, ny, nz, mean=synth.ARITH, dt=10.0, L=(64.0, 64.0, 64.0), bc=None):
    hx, hy, hz = (L[0] / (nx + 1), L[1] / (ny + 1), L[2] / (nz + 1))
    P = synth.Problem(nx=nx, ny=ny, nz=nz, hx=hx, hy=hy, hz=hz, mean=mean, dt=dt)
    if bc is not None:
        P.bc_type, P.bc_value = bc
    return P


def all_dirichlet(value_top=synth.P_TOP, value_other=synth.P_INIT):
    return ((synth.DIRICHLET,) * 6, (value_other,) * 5 + (value_top,))


def random_heads(n, seed, lo=-80.0, hi=-5.0, saturated_fraction=0.0):
    rng = np.random.default_rng(seed)
    p = rng.uniform(lo, hi, n)
    if saturated_fraction > 0:
        m = rng.random(n) < saturated_fraction
        p[m] = rng.uniform(0.0, 5.0, m.sum())
    return p


def random_ks(P, seed, sigma=1.5, ell=(2.0, 2.0, 1.0)):
    return synth.lognormal_ks((P.nx, P.ny, P.nz), synth.KS0, sigma, ell, seed)


def smooth_recipe(name, n, **kw):
    """A recipe at a reduced cube size (correlation lengths in cells unchanged)."""
    return synth.recipe(name, n=n, **kw) if name != "c1" else synth.recipe(name, n=n)


def random_spd_graph(n, density, seed):
    """A random symmetric M-matrix (negative off-diagonals, diagonally dominant) as CSR."""
    rng = np.random.default_rng(seed)
    A = sp.random(n, n, density=density, random_state=rng, format="coo")
    A = -(abs(A) + abs(A).T)
    A = sp.csr_matrix(A)
    A.setdiag(0)
    A.eliminate_zeros()
    d = -np.asarray(A.sum(axis=1)).ravel() + rng.uniform(0.01, 1.0, n)
    A = A + sp.diags(d)
    A = sp.csr_matrix(A)
    A.sort_indices()
    return A


def csr_close(rp1, c1, v1, A2, rtol):
    """Same pattern (bit-exact) and values within rtol of each row's largest entry."""
    A2 = sp.csr_matrix(A2)
    A2.sort_indices()
    assert np.array_equal(rp1, A2.indptr), "row pointers differ"
    assert np.array_equal(c1, A2.indices), "column indices differ"
    rowmax = np.maximum.reduceat(np.abs(A2.data), A2.indptr[:-1]) if A2.nnz else np.zeros(0)
    scale = np.repeat(rowmax, np.diff(A2.indptr))
    err = np.abs(v1 - A2.data)
    assert np.all(err <= rtol * scale), f"max scaled err {np.max(err / np.maximum(scale, 1e-300)):.3e}"
