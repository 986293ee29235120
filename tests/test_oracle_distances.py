"""Pins for the oracle's pairwise distances (the input step, Sec. 2.2).

Hamming: against the one-hot inner-product formulation of the input
generator (an independent evaluation: L - <onehot_i, onehot_j> as exact
float32 sums), brute force in pure Python on tiny inputs, the unknown-base
rule, and the metric axioms on the counts.  Euclidean: against the blocked
evaluation of the input generator (same roundings, other loop order over i),
closed forms (collinear points, Pythagorean triples), exact symmetry and a
zero diagonal, and scipy's cdist within a few ulps.
"""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import distances as OD


def test_hamming_matches_one_hot_formulation():
    reads, _ = W.amplicon_reads(300, 7, length=61, seed=4)
    for dt in (np.float32, np.float64):
        assert np.array_equal(OD.hamming(reads, dt), W.hamming_distances(reads, dt))


def test_hamming_brute_force_and_unknown_bases():
    rng = np.random.default_rng(1)
    codes = rng.integers(0, 4, size=(9, 13)).astype(np.uint8)
    codes[2, 5] = 4
    codes[7, 0] = 255
    D = OD.hamming(codes, np.float64)
    for i, j in itertools.product(range(9), repeat=2):
        c = sum(1 for p in range(13) if codes[i, p] != codes[j, p] or codes[i, p] > 3 or codes[j, p] > 3)
        assert D[i, j] == c / 13
    assert D[2, 2] == 1 / 13 and D[7, 7] == 1 / 13 and D[0, 0] == 0.0
    # float32: the float64 quotient rounded once; selected rows alone
    assert np.array_equal(OD.hamming(codes, np.float32), D.astype(np.float32))
    assert np.array_equal(OD.hamming(codes, np.float64, rows=[7, 2]), D[[7, 2]])


def test_hamming_counts_are_a_metric():
    reads, _ = W.amplicon_reads(60, 3, length=40, seed=2)
    C = np.rint(OD.hamming(reads, np.float64) * 40).astype(int)
    assert np.array_equal(C, C.T) and np.all(np.diag(C) == 0)
    assert np.all(C[:, :, None] <= C[:, None, :] + C.T[None, :, :])  # c_ik <= c_ij + c_jk


def test_euclidean_matches_blocked_recipe_and_closed_forms():
    X, _ = W.gaussian_mixture(257, 11, 4, 9.0, seed=3)
    for dt in (np.float32, np.float64):
        D = OD.euclidean(X, dt)
        assert np.array_equal(D, W.euclidean_distances(X, dt, block=64))
        assert np.array_equal(D, D.T) and np.all(np.diag(D) == 0)
    assert np.array_equal(OD.euclidean(X, np.float64, rows=[5, 0]), OD.euclidean(X, np.float64)[[5, 0]])
    x = np.array([[0.0], [1.5], [-2.25], [10.0]])
    assert np.array_equal(OD.euclidean(x, np.float64), np.abs(x - x.T))
    p = np.array([[0.0, 0.0], [3.0, 4.0], [-5.0, 12.0], [8.0, -15.0]])
    D = OD.euclidean(p, np.float64)
    assert D[0, 1] == 5.0 and D[0, 2] == 13.0 and D[0, 3] == 17.0


def test_euclidean_against_scipy_cdist():
    spatial = pytest.importorskip("scipy.spatial.distance")
    X, _ = W.gaussian_mixture(200, 23, 5, 4.0, seed=7)
    D = OD.euclidean(X, np.float64)
    ref = spatial.cdist(X, X)
    assert np.max(np.abs(D - ref) / np.maximum(ref, 1e-300)) < 8 * 2.0 ** -53
