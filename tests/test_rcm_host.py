"""The library's host reverse Cuthill-McKee ordering (bo_rcm, through the C
ABI; no GPU needed) against the oracle, bit for bit: road graphs of several
widths, a path, a star, several components, isolated nodes, self-loops and
repeated entries, n = 0 and n = 1; and its argument errors.  The permuted
pattern (bo_csr_permute) against SciPy's symmetric permutation of the sparse
matrix."""
import os

import numpy as np
import pytest

import oracle
from paper_1902_10078_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBPATH = os.path.join(ROOT, "paper_1902_10078_amd", "libbandops.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIBPATH), reason="libbandops.so not built")


def csr(n, edges, loops=(), repeats=()):
    rows, cols = [], []
    for a, b in list(edges) + list(repeats):
        rows += [a, b]
        cols += [b, a]
    for a in loops:
        rows.append(a)
        cols.append(a)
    rows, cols = np.array(rows, dtype=np.int64), np.array(cols, dtype=np.int64)
    o = np.lexsort((cols, rows))
    ip = np.zeros(n + 1, dtype=np.int64)
    np.add.at(ip, rows[o] + 1, 1)
    return np.cumsum(ip), cols[o]


def check(n, ip, ix):
    from paper_1902_10078_amd import bandops
    perm, iperm, bw = bandops.rcm(ip, ix)
    ref = oracle.rcm(n, ip, ix)
    assert np.array_equal(perm, ref)
    assert np.array_equal(iperm[perm], np.arange(n))
    assert bw == oracle.bandwidth(n, ip, ix, ref)


@pytest.mark.parametrize("W,L,seed", [(4, 300, 1), (6, 200, 2), (8, 100, 3), (3, 500, 4), (2, 50, 5)])
def test_rcm_road_graphs(W, L, seed):
    n, ip, ix, _ = inputs.road_graph(W, L, seed=seed)
    check(n, ip, ix)


def test_rcm_small_graphs():
    rng = np.random.default_rng(3)
    lab = rng.permutation(30)
    check(30, *csr(30, [(lab[i], lab[i + 1]) for i in range(29)]))
    check(9, *csr(9, [(4, j) for j in range(9) if j != 4]))
    check(8, *csr(8, [(5, 2), (2, 7), (0, 1), (1, 3), (3, 0), (3, 6)]))
    # self-loops, repeated entries and isolated nodes
    check(12, *csr(12, [(0, 5), (5, 9), (9, 1), (2, 3)], loops=(0, 5, 7, 11), repeats=((5, 9), (2, 3))))
    check(1, np.array([0, 0], dtype=np.int64), np.zeros(0, dtype=np.int64))
    # random sparse graph with many degree ties
    e = [(int(a), int(b)) for a, b in rng.integers(0, 200, size=(300, 2)) if a != b]
    check(200, *csr(200, e))


def test_rcm_empty_and_errors():
    import ctypes
    from paper_1902_10078_amd import bandops
    L = bandops.lib()
    ip = np.array([0], dtype=np.int64)
    hp = lambda a: ctypes.c_void_p(a.ctypes.data)
    assert L.bo_rcm(0, hp(ip), None, None, None, None) == 0
    bad = np.array([0, 2, 1], dtype=np.int64)   # decreasing indptr
    ix = np.array([1, 0], dtype=np.int64)
    perm = np.zeros(2, dtype=np.int64)
    assert L.bo_rcm(2, hp(bad), hp(ix), hp(perm), None, None) == -1
    assert b"malformed" in L.bo_last_error()
    out = np.array([0, 1, 2], dtype=np.int64)
    ix2 = np.array([5, 0], dtype=np.int64)      # index outside [0, n)
    assert L.bo_rcm(2, hp(out), hp(ix2), hp(perm), None, None) == -1


@pytest.mark.parametrize("W,L", [(4, 300), (3, 1000), (6, 50)])
def test_csr_permute_matches_scipy(W, L):
    import scipy.sparse as sp
    from paper_1902_10078_amd import bandops
    n, ip, ix, ln = inputs.road_graph(W, L, seed=W)
    qip, qix, qv = inputs.graph_gmrf_csr(n, ip, ix, ln)
    perm, iperm, _ = bandops.rcm(qip, qix)
    pip, pix, mp = bandops.csr_permute(qip, qix, perm, iperm)
    A = sp.csr_matrix((qv, qix, qip), shape=(n, n))[perm][:, perm].tocsr()
    A.sort_indices()
    assert np.array_equal(pip, A.indptr) and np.array_equal(pix, A.indices)
    assert np.array_equal(qv[mp], A.data)
    # an ordering that is not a permutation is refused
    import ctypes
    hp = lambda a: ctypes.c_void_p(a.ctypes.data)
    bad = perm.copy()
    bad[0] = bad[1]
    out = np.zeros(n + 1, dtype=np.int64)
    o2 = np.zeros(qix.size, dtype=np.int64)
    assert bandops.lib().bo_csr_permute(n, hp(qip), hp(qix), hp(bad), hp(iperm), hp(out), hp(o2), hp(o2)) == -1
