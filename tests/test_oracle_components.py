"""Pins for the oracle's threshold-graph components (Sec. 7, Conclusions and
perspectives): against scipy's connected_components (an independent
library), a breadth-first search in pure Python on tiny graphs, the empty and
the complete graph, NaN entries, the full-matrix reading of an asymmetric D,
the row-block form, and planted clusters whose components are known."""
import collections

import numpy as np
import pytest

import workloads as W
from oracle import components as OC


def canonical(labels):
    lab = np.asarray(labels)
    first = {}
    for v, r in enumerate(lab):
        first.setdefault(int(r), v)
    return np.array([first[int(r)] for r in lab], dtype=np.int32)


def bfs_components(adj):
    n = len(adj)
    lab = [-1] * n
    for s in range(n):
        if lab[s] >= 0:
            continue
        lab[s] = s
        q = collections.deque([s])
        while q:
            u = q.popleft()
            for v in adj[u]:
                if lab[v] < 0:
                    lab[v] = s
                    q.append(v)
    return np.array(lab, dtype=np.int32)


def random_symmetric(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.random((n, n))
    D = np.triu(A, 1)
    D = D + D.T
    return D


@pytest.mark.parametrize("n,theta", [(1, 0.5), (2, 0.3), (9, 0.15), (40, 0.03), (120, 0.012), (300, 0.004)])
def test_components_match_bfs_and_scipy(n, theta):
    csgraph = pytest.importorskip("scipy.sparse.csgraph")
    sparse = pytest.importorskip("scipy.sparse")
    D = random_symmetric(n, seed=n)
    lab, cnt = OC.threshold_components(D, theta)
    adj = [[j for j in range(n) if j != i and D[i, j] <= theta] for i in range(n)]
    assert np.array_equal(lab, bfs_components(adj))
    A = sparse.csr_matrix(np.triu(D <= theta, 1))
    k, sl = csgraph.connected_components(A, directed=False)
    assert cnt == k and np.array_equal(lab, canonical(sl))
    assert np.all(lab <= np.arange(n)) and np.array_equal(lab[lab], lab)


def test_empty_complete_and_nan():
    D = random_symmetric(50, seed=3)
    lab, cnt = OC.threshold_components(D, -1.0)
    assert cnt == 50 and np.array_equal(lab, np.arange(50))
    lab, cnt = OC.threshold_components(D, 2.0)
    assert cnt == 1 and np.all(lab == 0)
    Dn = D.copy()
    Dn[:, 7] = np.nan
    Dn[7, :] = np.nan
    lab, cnt = OC.threshold_components(Dn, 2.0)
    assert cnt == 2 and lab[7] == 7 and np.all(np.delete(lab, 7) == 0)


def test_full_matrix_reads_both_triangles():
    D = np.full((4, 4), 9.0)
    np.fill_diagonal(D, 0.0)
    D[2, 0] = 1.0  # below the diagonal only
    D[1, 3] = 1.0  # above the diagonal only
    lab, cnt = OC.threshold_components(D, 1.0)
    assert list(lab) == [0, 1, 2, 1] and cnt == 3
    lab, cnt = OC.threshold_components(D, 1.0, full=True)
    assert list(lab) == [0, 1, 0, 1] and cnt == 2


def test_row_blocks_equal_whole_matrix():
    D = random_symmetric(200, seed=9)
    want = OC.threshold_components(D, 0.01)
    blocks = [(a, D[a:a + 37]) for a in range(0, 200, 37)]
    got = OC.threshold_components_rows(200, 0.01, blocks)
    assert np.array_equal(got[0], want[0]) and got[1] == want[1]


def test_planted_clusters():
    # reads of distinct random references: within a reference the distances
    # are at most about twice the substitution rate, between references
    # about 3/4; a threshold between them recovers the references
    reads, parent = W.amplicon_reads(400, 6, rate_lo=0.01, rate_hi=0.02, length=300, seed=1)
    D = W.hamming_distances(reads)
    lab, cnt = OC.threshold_components(D, 0.2)
    assert cnt == len(np.unique(parent))
    assert np.array_equal(lab, canonical(parent))
