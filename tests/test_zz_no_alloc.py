"""rich_match_sweep_noalloc (the matching sweep for callers that cannot
allocate) against rich_match_sweep through the C-ABI: the same aggregates and
coarse size bit for bit, on two calls in a row with the second input smaller
than the first (the shared work array keeps the first call's contents), and a
clear error for an input beyond the array."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from tests.helpers import box_problem, random_heads, random_ks, random_spd_graph

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


def _dev(torch, A):
    A = sp.csr_matrix(A)
    A.sort_indices()
    return (torch.from_numpy(A.indptr.astype(np.int64)).cuda(), torch.from_numpy(A.indices.astype(np.int32)).cuda(),
            torch.from_numpy(A.data.astype(np.float64)).cuda())


def _both(rich, torch, A):
    rp, col, val = _dev(torch, A)
    agg_ref, nc_ref = rich.match_sweep(rp, col, val)
    out = torch.full((A.shape[0],), -7, dtype=torch.int32, device="cuda")
    agg, nc = rich.match_sweep(rp, col, val, agg=out, noalloc=True)
    return agg_ref.cpu().numpy(), nc_ref, agg.cpu().numpy(), nc


def test_noalloc_sweep_equals_the_allocating_one(rich, torch, orc):
    # a grid's auxiliary matrix (64,000 rows), then a smaller random graph with
    # exact weight ties, then the grid again
    P = box_problem(40, 40, 40, mean=synth.UPSTREAM)
    M = orc.auxiliary(P, random_ks(P, 3), random_heads(P.n, 4, -70, -30))
    T = random_spd_graph(3000, 0.002, 5)
    T.data = np.round(T.data * 2) / 2
    T.data[T.data == 0] = -0.5
    T.setdiag(np.abs(T.diagonal()) + 1.0)
    for A in (M, T, M):
        a_ref, nc_ref, a, nc = _both(rich, torch, A)
        assert nc == nc_ref and 0 < nc < A.shape[0]
        assert np.array_equal(a, a_ref)


def test_noalloc_sweep_rejects_inputs_beyond_its_array(rich, torch):
    from paper_2112_05051_amd import _lib
    n = 2_500_000  # 32 n + 8 nnz bytes > 64 MiB
    A = sp.identity(n, format="csr") * 2.0
    rp, col, val = _dev(torch, A)
    with pytest.raises(_lib.RichError) as e:
        rich.match_sweep(rp, col, val, noalloc=True)
    assert e.value.status == _lib.EBUDGET
    del rp, col, val
    # still usable afterwards
    T = random_spd_graph(500, 0.02, 6)
    a_ref, nc_ref, a, nc = _both(rich, torch, T)
    assert nc == nc_ref and np.array_equal(a, a_ref)
