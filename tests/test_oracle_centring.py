"""Pins for the oracle's double centring (Sec. 6.2, step 1).

Independent checks: the Gram matrix of a Euclidean point cloud equals the
inner products of the centred points (what the equation is derived from), the
matrix form -1/2 J D^2 J, vanishing row/column sums, the trace identity and
exact (fsum) means.
"""
import math

import numpy as np

import oracle as O
import workloads as W


def test_gram_equals_centred_inner_products():
    X, _ = W.gaussian_mixture(120, 7, 3, 25.0, seed=3)
    D = W.euclidean_distances(X)
    G = O.gram_matrix(D)
    Xc = X - X.mean(axis=0)
    ref = Xc @ Xc.T
    assert np.max(np.abs(G - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_matrix_form_with_centring_operator_nonsymmetric():
    rng = np.random.default_rng(4)
    n = 33
    D = rng.random((n, n)) * 3.0  # deliberately not symmetric
    J = np.eye(n) - np.ones((n, n)) / n
    ref = -0.5 * J @ (D * D) @ J
    assert np.max(np.abs(O.gram_matrix(D) - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_rows_and_columns_sum_to_zero_and_trace():
    reads, _ = W.amplicon_reads(200, 6, seed=1)
    D = W.hamming_distances(reads)
    G = O.gram_matrix(D)
    scale = np.abs(G).sum(axis=1)
    assert np.all(np.abs(G.sum(axis=1)) <= 1e-13 * scale)
    assert np.all(np.abs(G.sum(axis=0)) <= 1e-13 * np.abs(G).sum(axis=0))
    D64 = D.astype(np.float64)
    n = D.shape[0]
    # trace identity for a symmetric D with zero diagonal: tr G = sum d^2 / (2n)
    assert math.isclose(np.trace(G), (D64 ** 2).sum() / (2 * n), rel_tol=1e-13)


def test_stats_against_exact_sums():
    rng = np.random.default_rng(8)
    D = rng.random((17, 17)).astype(np.float32)
    r, c, m = O.centring_stats(D)
    D2 = [[float(x) ** 2 for x in row] for row in D.astype(np.float64)]
    n = 17
    for i in range(n):
        assert math.isclose(r[i], math.fsum(D2[i]) / n, rel_tol=1e-15)
        assert math.isclose(c[i], math.fsum(D2[j][i] for j in range(n)) / n, rel_tol=1e-15)
    assert math.isclose(m, math.fsum(v for row in D2 for v in row) / n ** 2, rel_tol=1e-15)


def test_sampled_entries_match_full_matrix():
    rng = np.random.default_rng(2)
    D = rng.random((40, 40))
    D = D + D.T
    np.fill_diagonal(D, 0)
    r, c, m = O.centring_stats(D)
    G = O.gram_matrix(D)
    ii = rng.integers(0, 40, 25)
    jj = rng.integers(0, 40, 25)
    assert np.allclose(O.gram_entries(D[ii, jj], r[ii], c[jj], m), G[ii, jj], rtol=0, atol=1e-14)
