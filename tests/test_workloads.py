"""Checks of the synthetic input generators (not part of the method)."""
import numpy as np

import workloads as W


def test_hamming_counts_brute_force():
    reads, parent = W.amplicon_reads(40, 3, seed=0, length=70)
    c = W.hamming_counts(reads)
    for i in range(40):
        for j in range(40):
            assert c[i, j] == int(np.sum(reads[i] != reads[j]))
    assert np.all(np.diag(c) == 0) and np.array_equal(c, c.T)


def test_amplicon_recipe_properties():
    reads, parent = W.amplicon_reads(3000, 5, seed=1)
    assert reads.dtype == np.uint8 and reads.max() <= 3
    assert set(np.unique(parent)) == set(range(5))
    D = W.hamming_distances(reads[:300])
    assert D.dtype == np.float32
    same = parent[:300, None] == parent[None, :300]
    off = ~np.eye(300, dtype=bool)
    # within-reference distances about 2 x 1-5 % substitutions, across about 3/4
    assert 0.01 < D[same & off].mean() < 0.1
    assert 0.7 < D[~same].mean() < 0.8
    assert np.array_equal(W.amplicon_reads(50, 5, seed=1)[0], W.amplicon_reads(50, 5, seed=1)[0])


def test_hamming_distance_rounding_rule():
    reads, _ = W.amplicon_reads(30, 2, seed=2)
    c = W.hamming_counts(reads)
    D = W.hamming_distances(reads)
    assert np.array_equal(D, (c.astype(np.float64) / 400.0).astype(np.float32))


def test_bitplanes_encode_reads():
    reads, _ = W.amplicon_reads(9, 2, seed=3)
    P = W.pack_bitplanes(reads)
    assert P.shape == (9, 4, 7)
    for i in range(9):
        for b in range(4):
            for t in range(400):
                bit = (int(P[i, b, t // 64]) >> (t % 64)) & 1
                assert bit == int(reads[i, t] == b)
    # pad bits beyond the read length are zero
    assert all((int(P[i, b, 6]) >> 16) == 0 for i in range(9) for b in range(4))


def test_gaussian_mixture_and_distances():
    X, lab = W.gaussian_mixture(50, 4, 3, 25.0, seed=0)
    X2, _ = W.gaussian_mixture(50, 4, 3, 25.0, seed=0)
    assert np.array_equal(X, X2)
    D = W.euclidean_distances(X, block=7)
    assert np.all(np.diag(D) == 0) and np.array_equal(D, D.T)
    i, j = 3, 41
    assert np.isclose(D[i, j], np.sqrt(np.sum((X[i] - X[j]) ** 2)), rtol=1e-15)
    D32 = W.euclidean_distances(X, dtype=np.float32)
    assert np.array_equal(D32, D.astype(np.float32))
