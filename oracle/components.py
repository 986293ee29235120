"""Plain CPU oracle of the threshold-graph components (Sec. 7, Conclusions
and perspectives: vertices are the items, (i, j) is an edge iff
d(i, j) <= theta, and the connected components of that graph are formed).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Union-find over the
edges in row order, written out plainly; the result is reported in the
canonical form labels[i] = smallest index in the component of i, which does
not depend on how the components were found.

By default only the upper triangle j > i of D is examined (D symmetric by
contract); with ``full=True`` an edge exists iff d_ij <= theta or
d_ji <= theta.  Each entry is compared as a float64 value; NaN is no edge.
``threshold_components_rows`` takes D as consecutive row blocks (for D that
lives elsewhere and is fetched block by block), default mode only.
"""
from __future__ import annotations

import numpy as np

__all__ = ["threshold_components", "threshold_components_rows"]


class _Forest:
    def __init__(self, n: int):
        self.parent = list(range(n))

    def find(self, v: int) -> int:
        root = v
        while self.parent[root] != root:
            root = self.parent[root]
        while self.parent[v] != root:  # compress the path
            self.parent[v], v = root, self.parent[v]
        return root

    def union(self, a: int, b: int) -> None:
        ra, rb = self.find(a), self.find(b)
        if ra != rb:
            self.parent[max(ra, rb)] = min(ra, rb)

    def labels(self) -> np.ndarray:
        n = len(self.parent)
        lab = np.array([self.find(v) for v in range(n)], dtype=np.int64)
        # canonical form: the smallest member of each component
        smallest = {}
        for v in range(n):
            smallest.setdefault(int(lab[v]), v)
        return np.array([smallest[int(r)] for r in lab], dtype=np.int32)


def threshold_components(D: np.ndarray, theta: float, full: bool = False):
    D = np.asarray(D)
    n = D.shape[0]
    f = _Forest(n)
    for i in range(n):
        row = D[i].astype(np.float64)
        edge = row <= theta
        if full:
            edge |= D[:, i].astype(np.float64) <= theta
        edge[: i + 1] = False  # each unordered pair once (j > i)
        for j in np.nonzero(edge)[0]:
            f.union(i, int(j))
    lab = f.labels()
    return lab, int(np.sum(lab == np.arange(n)))


def threshold_components_rows(n: int, theta: float, blocks):
    """Same as the default mode of ``threshold_components`` with D given as
    an iterable of (first_row, rows) blocks covering rows 0..n-1 in order."""
    f = _Forest(n)
    for r0, rows in blocks:
        rows = np.asarray(rows, dtype=np.float64)
        for a in range(rows.shape[0]):
            i = r0 + a
            js = np.nonzero(rows[a, i + 1:] <= theta)[0] + i + 1
            for j in js:
                f.union(i, int(j))
    lab = f.labels()
    return lab, int(np.sum(lab == np.arange(n)))
