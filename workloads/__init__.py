"""Seeded synthetic inputs for random-projection classical MDS.

These generators stand in for the Lake Geneva rbcL amplicon samples of the
paper (Sec. 6.1; L6 with about 1e5 reads in Sec. 4.1), which are not
available.  They produce distance matrices only: nothing here performs any
step of the MDS method itself (no squaring, centring, projection or
eigensolve), so both the oracle and the GPU library may consume their output.

Two families:

* Gaussian-mixture point clouds with Euclidean distances (the case where the
  Gram matrix is positive semi-definite, Sec. 6.3).
* Amplicon-like reads: random ACGT references of length 400 and reads that
  copy one reference with i.i.d. substitutions; the distance is the Hamming
  count divided by the read length (a stand-in for the alignment-based
  dissimilarity of Sec. 2.2).  Such a D is generally not Euclidean.

All randomness comes from ``numpy.random.default_rng(seed)`` in a fixed
draw order, so a (recipe, seed) pair names one input exactly.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gaussian_mixture",
    "euclidean_distances",
    "amplicon_reads",
    "hamming_counts",
    "hamming_distances",
    "pack_bitplanes",
    "ReadsRecipe",
]

READ_LENGTH = 400


def gaussian_mixture(n: int, dim: int, n_comp: int, mean_var: float, seed: int):
    """Points x_i = mu_{z_i} + e_i, mu_c ~ N(0, mean_var I), e_i ~ N(0, I),
    z_i uniform over the n_comp components.

    Draw order: means (n_comp x dim), labels (n), noise (n x dim).
    Returns (X float64 n x dim, labels int64 n).
    """
    rng = np.random.default_rng(seed)
    means = rng.normal(0.0, np.sqrt(mean_var), size=(n_comp, dim))
    labels = rng.integers(0, n_comp, size=n)
    noise = rng.standard_normal(size=(n, dim))
    return means[labels] + noise, labels


def euclidean_distances(X: np.ndarray, dtype=np.float64, block: int = 512) -> np.ndarray:
    """d_ij = sqrt(sum_k (x_ik - x_jk)^2), accumulated in float64 over k in
    increasing order (direct differences, no Gram shortcut), then rounded to
    ``dtype``.  The diagonal is exactly zero and D is exactly symmetric."""
    X = np.asarray(X, dtype=np.float64)
    n, dim = X.shape
    D = np.empty((n, n), dtype=dtype)
    for a in range(0, n, block):
        b = min(a + block, n)
        acc = np.zeros((b - a, n), dtype=np.float64)
        for k in range(dim):
            diff = X[a:b, k][:, None] - X[None, :, k]
            acc += diff * diff
        D[a:b] = np.sqrt(acc).astype(dtype)
    return D


class ReadsRecipe:
    """Parameters of the amplicon-read generator."""

    def __init__(self, n_reads: int, n_refs: int, rate_lo: float = 0.01,
                 rate_hi: float = 0.05, length: int = READ_LENGTH, seed: int = 0):
        self.n_reads = int(n_reads)
        self.n_refs = int(n_refs)
        self.rate_lo = float(rate_lo)
        self.rate_hi = float(rate_hi)
        self.length = int(length)
        self.seed = int(seed)


def amplicon_reads(n_reads: int, n_refs: int, rate_lo: float = 0.01,
                   rate_hi: float = 0.05, length: int = READ_LENGTH, seed: int = 0):
    """Reads over the alphabet {0,1,2,3} (A,C,G,T).

    References: i.i.d. uniform bases.  Each read copies a uniformly chosen
    reference; its substitution rate rho ~ U[rate_lo, rate_hi]; each site is
    substituted independently with probability rho by one of the three other
    bases, chosen uniformly.

    Draw order: refs (n_refs x L), parent (n), rho (n), site uniforms (n x L),
    base shifts (n x L).  Returns (reads uint8 n x L, parent int64 n).
    """
    rng = np.random.default_rng(seed)
    refs = rng.integers(0, 4, size=(n_refs, length), dtype=np.uint8)
    parent = rng.integers(0, n_refs, size=n_reads)
    rho = rng.uniform(rate_lo, rate_hi, size=n_reads)
    reads = refs[parent].copy()
    # generate the per-site draws in row chunks to bound memory at large n
    chunk = 8192
    for a in range(0, n_reads, chunk):
        b = min(a + chunk, n_reads)
        site = rng.random(size=(b - a, length))
        shift = rng.integers(1, 4, size=(b - a, length), dtype=np.uint8)
        sub = site < rho[a:b, None]
        blk = reads[a:b]
        reads[a:b] = np.where(sub, (blk + shift) % 4, blk).astype(np.uint8)
    return reads, parent


def hamming_counts(reads: np.ndarray, block: int = 2048) -> np.ndarray:
    """Exact integer mismatch counts between all pairs of reads (int32 n x n),
    via one-hot encodings: matches = <onehot_i, onehot_j>, counts = L - matches.
    The float32 products are sums of at most L ones, hence exact."""
    reads = np.asarray(reads, dtype=np.uint8)
    n, L = reads.shape
    oh = np.zeros((n, 4 * L), dtype=np.float32)
    oh[np.arange(n)[:, None], np.arange(L)[None, :] * 4 + reads] = 1.0
    out = np.empty((n, n), dtype=np.int32)
    for a in range(0, n, block):
        b = min(a + block, n)
        out[a:b] = L - (oh[a:b] @ oh.T).astype(np.int32)
    return out


def hamming_distances(reads: np.ndarray, dtype=np.float32) -> np.ndarray:
    """d_ij = count_ij / L, evaluated as a float64 division and then rounded
    to ``dtype`` (round-to-nearest-even).  The GPU generator uses the same
    two roundings, so both produce identical bits."""
    reads = np.asarray(reads)
    L = reads.shape[1]
    c = hamming_counts(reads)
    return (c.astype(np.float64) / float(L)).astype(dtype)


def pack_bitplanes(reads: np.ndarray) -> np.ndarray:
    """One bit-plane per base: planes[i, b, w] has bit t set iff
    reads[i, 64*w + t] == b.  Shape (n, 4, ceil(L/64)) uint64, used by the
    GPU Hamming generator."""
    reads = np.asarray(reads, dtype=np.uint8)
    n, L = reads.shape
    words = (L + 63) // 64
    planes = np.zeros((n, 4, words), dtype=np.uint64)
    for b in range(4):
        bits = (reads == b)
        padded = np.zeros((n, words * 64), dtype=bool)
        padded[:, :L] = bits
        # little-endian bit order inside each 64-bit word
        by = np.packbits(padded.reshape(n, words, 8, 8), axis=-1, bitorder="little")
        planes[:, b, :] = by.reshape(n, words, 8).view(np.uint64).reshape(n, words)
    return planes
