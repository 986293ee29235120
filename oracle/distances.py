"""Plain CPU oracle of the pairwise distances (Sec. 2.2: the dissimilarity
matrix D between reads that the method takes as input; Table 1 lists its
computation as the pipeline's dominant cost).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Written from the
definitions, one output row at a time, with no blocking or reformulation:

* ``hamming``: d_ij = (number of positions at which the base codes of reads i
  and j differ) / L, the float64 quotient rounded to the output type.  A
  code outside 0..3 (an unknown base) counts as a mismatch against every
  code, itself included.  Substitution-only reads stand in for the
  alignment-based dissimilarity of Sec. 2.2.
* ``euclidean``: d_ij = sqrt(sum_k (x_ik - x_jk)^2) with the square and each
  partial sum rounded to float64, k increasing, the square root rounded to
  float64 and then to the output type.
"""
from __future__ import annotations

import numpy as np

__all__ = ["hamming", "euclidean"]


def hamming(codes: np.ndarray, dtype=np.float32, rows=None) -> np.ndarray:
    """The n x n matrix, or only the listed rows (len(rows) x n)."""
    codes = np.asarray(codes, dtype=np.uint8)
    n, L = codes.shape
    rows = np.arange(n) if rows is None else np.asarray(rows)
    unknown = codes > 3
    D = np.empty((len(rows), n), dtype=dtype)
    for a, i in enumerate(rows):
        differ = (codes[i][None, :] != codes) | unknown[i][None, :] | unknown
        count = differ.sum(axis=1)  # exact integers
        D[a] = (count.astype(np.float64) / float(L)).astype(dtype)
    return D


def euclidean(X: np.ndarray, dtype=np.float32, rows=None) -> np.ndarray:
    """The n x n matrix, or only the listed rows (len(rows) x n)."""
    X = np.asarray(X, dtype=np.float64)
    n, dim = X.shape
    rows = np.arange(n) if rows is None else np.asarray(rows)
    D = np.empty((len(rows), n), dtype=dtype)
    for a, i in enumerate(rows):
        acc = np.zeros(n, dtype=np.float64)
        for k in range(dim):
            d = X[i, k] - X[:, k]
            sq = d * d
            acc = acc + sq
        D[a] = np.sqrt(acc).astype(dtype)
    return D
