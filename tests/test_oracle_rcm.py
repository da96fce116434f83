"""Pins for the oracle's reverse Cuthill-McKee ordering and band assembly of a
GMRF precision on a graph (Section 2; the ordering Section 5 uses for its
road-network GMRF).

- Closed forms: a path graph in a random labelling comes back as the path
  (bandwidth 1), a star as leaf, centre, leaves, two components one after the
  other; the order is the reverse of a breadth-first traversal whose levels,
  start nodes and sibling order satisfy the Cuthill-McKee rule.
- SciPy's `reverse_cuthill_mckee`: the same permutation on a road graph
  whose traversal has no ties that the two tie-breaking rules resolve
  differently, and comparable bandwidths on larger ones.
- Reversal matters: the envelope (profile) of the reversed order is no larger
  than that of the unreversed Cuthill-McKee order.
- Band assembly against the dense permuted matrix (numpy); the synthetic
  graph precision is symmetric positive definite."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee

import oracle
from bandutil import dense_to_lower
from paper_1902_10078_amd import inputs


def csr_of_edges(n, edges):
    A = sp.lil_matrix((n, n))
    for a, b in edges:
        A[a, b] = A[b, a] = 1.0
    A = A.tocsr()
    A.sort_indices()
    return A.indptr.astype(np.int64), A.indices.astype(np.int64)


def test_path_graph_comes_back_as_a_path():
    rng = np.random.default_rng(1)
    n = 40
    lab = rng.permutation(n)
    ip, ix = csr_of_edges(n, [(lab[i], lab[i + 1]) for i in range(n - 1)])
    p = oracle.rcm(n, ip, ix)
    assert oracle.bandwidth(n, ip, ix, p) == 1
    # Cuthill-McKee starts at the endpoint with the lower label and walks the path
    start = min(lab[0], lab[-1])
    walk = list(lab) if start == lab[0] else list(lab[::-1])
    assert list(p) == walk[::-1]


def test_star_graph():
    n = 9
    ip, ix = csr_of_edges(n, [(4, j) for j in range(n) if j != 4])
    p = oracle.rcm(n, ip, ix)
    # CM: lowest-degree node 0, then the centre 4, then the other leaves by index
    assert list(p) == [8, 7, 6, 5, 3, 2, 1, 4, 0]


def test_components_follow_their_lowest_degree_nodes():
    # component A: path 5-2-7; component B: triangle 0-1-3 with tail 3-6; node 4 isolated
    n = 8
    ip, ix = csr_of_edges(n, [(5, 2), (2, 7), (0, 1), (1, 3), (3, 0), (3, 6)])
    p = oracle.rcm(n, ip, ix)
    # degrees: 4:0, 5:1, 7:1, 6:1, 2:2, 0:2, 1:2, 3:3 -> CM: 4 | 5 2 7 | 6 3 0 1
    assert list(p) == [1, 0, 3, 6, 7, 2, 5, 4]


def cm_invariants(n, ip, ix, order):
    """Check the Cuthill-McKee rule on the unreversed order."""
    adj = [set(int(j) for j in ix[ip[i]:ip[i + 1]] if j != i) for i in range(n)]
    deg = [len(a) for a in adj]
    pos = {v: t for t, v in enumerate(order)}
    assert sorted(order) == list(range(n))
    # each node after a component's start is a child of its earliest-placed neighbour
    parent = {}
    for v in order:
        earlier = [u for u in adj[v] if pos[u] < pos[v]]
        if earlier:
            parent[v] = min(earlier, key=lambda u: pos[u])
        else:   # a component's start: no unvisited node of lower (degree, index) remains
            rest = [u for u in range(n) if pos[u] >= pos[v]]
            assert (deg[v], v) == min((deg[u], u) for u in rest)
    # children of one parent are consecutive and ordered by (degree, index); parents in visit order
    kids = {}
    for v in order:
        if v in parent:
            kids.setdefault(parent[v], []).append(v)
    for u, ch in kids.items():
        ps = [pos[c] for c in ch]
        assert ps == list(range(ps[0], ps[0] + len(ch)))
        assert [(deg[c], c) for c in ch] == sorted((deg[c], c) for c in ch)
    firsts = sorted(kids, key=lambda u: pos[u])
    assert [pos[kids[u][0]] for u in firsts] == sorted(pos[kids[u][0]] for u in firsts)


@pytest.mark.parametrize("W,L,seed", [(4, 60, 1), (6, 40, 2), (3, 200, 3), (8, 30, 4)])
def test_road_graph_order_satisfies_cuthill_mckee(W, L, seed):
    n, ip, ix, _ = inputs.road_graph(W, L, seed=seed)
    p = oracle.rcm(n, ip, ix)
    cm_invariants(n, ip, ix, list(p[::-1]))


def envelope(n, ip, ix, perm):
    inv = np.argsort(perm)
    first = np.arange(n)
    for i in range(n):
        for j in ix[ip[i]:ip[i + 1]]:
            a, b = inv[i], inv[j]
            if b < a:
                first[a] = min(first[a], b)
    return int(np.sum(np.arange(n) - first))


@pytest.mark.parametrize("W,L", [(4, 100), (6, 60), (8, 40)])
def test_reversal_does_not_enlarge_the_envelope(W, L):
    n, ip, ix, _ = inputs.road_graph(W, L, seed=W)
    p = oracle.rcm(n, ip, ix)
    assert envelope(n, ip, ix, p) <= envelope(n, ip, ix, p[::-1])


def test_same_permutation_as_scipy_without_tie_differences():
    n, ip, ix, _ = inputs.road_graph(4, 50)
    A = sp.csr_matrix((np.ones(len(ix)), ix, ip), shape=(n, n))
    assert np.array_equal(oracle.rcm(n, ip, ix), reverse_cuthill_mckee(A, symmetric_mode=True))


@pytest.mark.parametrize("W,L", [(4, 500), (6, 300), (8, 200), (3, 1000)])
def test_bandwidth_comparable_to_scipy(W, L):
    n, ip, ix, _ = inputs.road_graph(W, L, seed=7)
    A = sp.csr_matrix((np.ones(len(ix)), ix, ip), shape=(n, n))
    ours = oracle.bandwidth(n, ip, ix, oracle.rcm(n, ip, ix))
    ref = oracle.bandwidth(n, ip, ix, reverse_cuthill_mckee(A, symmetric_mode=True))
    assert ours <= 2 * ref and ours < oracle.bandwidth(n, ip, ix) / 10


def test_band_assembly_matches_dense_permutation():
    n, ip, ix, ln = inputs.road_graph(4, 30, seed=5)
    qip, qix, qv = inputs.graph_gmrf_csr(n, ip, ix, ln)
    p = oracle.rcm(n, qip, qix)
    k = oracle.bandwidth(n, qip, qix, p)
    B, dropped = oracle.csr_to_band(n, qip, qix, qv, p, k)
    assert dropped == 0
    Q = sp.csr_matrix((qv, qix, qip), shape=(n, n)).toarray()
    assert np.array_equal(B, dense_to_lower(Q[np.ix_(p, p)], k))
    # a narrower band drops exactly the entries outside it (each counted once, lower side)
    B2, dropped2 = oracle.csr_to_band(n, qip, qix, qv, p, k - 2)
    P = Q[np.ix_(p, p)]
    ii, jj = np.nonzero(np.tril(P, -(k - 1)))
    assert dropped2 == len(ii)
    assert np.allclose(Q, Q.T) and np.linalg.eigvalsh(Q).min() > 0
