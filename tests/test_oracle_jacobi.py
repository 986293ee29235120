"""Pins for the oracle's cyclic Jacobi eigensolver (``jacobi_eigh``) and for
exact classical MDS through it (Sec. 6.2, steps 2-3, for small n).

The pins are independent of the solver's own steps: a matrix built as
Q diag(lambda) Q^T from a chosen spectrum (repeated and negative values
included), the closed form of a 2 x 2 symmetric eigenproblem, the
eigen-residual and orthogonality of the vectors, and, for a Euclidean point
cloud, the squared singular values of the centred cloud (Sec. 6.3).
"""
import numpy as np

import oracle as O
import workloads as W


def _spectrum_matrix(lam, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((len(lam), len(lam))))
    return Q @ np.diag(lam) @ Q.T


def test_jacobi_recovers_a_chosen_spectrum():
    lam = np.array([7.5, 3.0, 3.0, 1.25, 0.0, 0.0, -0.5, -2.0, -2.0, -9.0, 4.0, 0.125])
    A = _spectrum_matrix(lam, 3)
    A = 0.5 * (A + A.T)
    w, V = O.jacobi_eigh(A)
    assert np.max(np.abs(w - np.sort(lam)[::-1])) <= 1e-13 * np.max(np.abs(lam))
    assert np.max(np.abs(V.T @ V - np.eye(len(lam)))) < 1e-13
    assert np.max(np.abs(A @ V - V * w[None, :])) < 1e-12 * np.max(np.abs(lam))


def test_jacobi_two_by_two_closed_form():
    for a, b, d in [(2.0, 1.0, -3.0), (1.0, 0.0, 1.0), (0.0, 5.0, 0.0), (1e-3, 2.0, 1e3)]:
        w, V = O.jacobi_eigh(np.array([[a, b], [b, d]]))
        mid, rad = 0.5 * (a + d), np.hypot(0.5 * (a - d), b)
        assert np.allclose(w, [mid + rad, mid - rad], rtol=1e-14, atol=1e-14 * (abs(mid) + rad))
        assert np.allclose(np.array([[a, b], [b, d]]) @ V, V * w[None, :], atol=1e-13 * (abs(mid) + rad))


def test_jacobi_diagonal_input_needs_no_rotation():
    w, V = O.jacobi_eigh(np.diag([1.0, 4.0, -2.0, 4.0]))
    assert np.array_equal(w, [4.0, 4.0, 1.0, -2.0])
    assert np.array_equal(np.abs(V), np.eye(4)[:, [1, 3, 0, 2]])


def test_full_mds_by_jacobi_matches_the_cloud_spectrum():
    X, _ = W.gaussian_mixture(48, 5, 3, 16.0, seed=2)
    D = W.euclidean_distances(X)
    Xc = X - X.mean(axis=0, keepdims=True)
    sig2 = np.sort(np.linalg.svd(Xc, compute_uv=False) ** 2)[::-1]
    res = O.full_mds(D, 5, method="jacobi")
    assert np.max(np.abs(res["eigvals"] - sig2) / sig2) < 1e-12
    assert np.max(np.abs(res["eigvals_all"][5:])) < 1e-10 * sig2[0]  # rank(G) = 5
    # the embedding reproduces D (k = rank), and agrees with the LAPACK route
    C = res["coords"]
    # (squared distances: the error of a small d grows like 1 / d after the root)
    dh2 = ((C[:, None, :] - C[None, :, :]) ** 2).sum(-1)
    assert np.max(np.abs(dh2 - D * D)) < 1e-11 * np.max(D * D)
    ref = O.full_mds(D, 5)
    assert np.max(np.abs(res["eigvals"] - ref["eigvals"]) / ref["eigvals"]) < 1e-12
