"""Pins for the oracle's exact and randomized classical MDS.

Exact MDS (Sec. 6.2 steps 2-3) is pinned by the Euclidean closed form
(eigenvalues = squared singular values of the centred cloud, Sec. 6.3's PCA
equivalence), by the embedding reproducing D, and by the projection identities
of a truncated embedding.  Randomized MDS (Sec. 3.2-3.3) is pinned by the
exactness of the range finder when rank(G) <= l, Cauchy interlacing,
convergence in q, the number of applications of G, and Rayleigh-Ritz
residuals.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle as O
import workloads as W


def _pdist(X):
    diff = X[:, None, :] - X[None, :, :]
    return np.sqrt((diff ** 2).sum(-1))


@pytest.fixture(scope="module")
def cloud():
    X, _ = W.gaussian_mixture(300, 6, 4, 25.0, seed=0)
    return X, W.euclidean_distances(X)


def test_full_mds_euclidean_closed_form(cloud):
    X, D = cloud
    res = O.full_mds(D, 6)
    s = np.linalg.svd(X - X.mean(axis=0), compute_uv=False)
    lam = res["eigvals_all"]
    assert np.allclose(lam[:6], s ** 2, rtol=1e-11, atol=0)
    assert np.max(np.abs(lam[6:])) <= 1e-9 * lam[0]
    # scipy/LAPACK symmetric eigensolver agrees on the spectrum
    ref = scipy.linalg.eigh(res["G"], eigvals_only=True)[::-1]
    assert np.allclose(lam, ref, rtol=0, atol=1e-12 * lam[0])


def test_full_embedding_reproduces_distances(cloud):
    _, D = cloud
    Xk = O.full_mds(D, 6)["coords"]
    assert np.max(np.abs(_pdist(Xk) - D)) <= 1e-9 * D.max()


def test_truncated_embedding_projection_identities(cloud):
    _, D = cloud
    n = D.shape[0]
    res = O.full_mds(D, 3)
    Dh = _pdist(res["coords"])
    assert np.all(Dh <= D + 1e-9 * D.max())  # orthogonal projection shrinks distances
    lost = (D ** 2 - Dh ** 2).sum()
    assert np.isclose(lost, 2 * n * res["eigvals_all"][3:].sum(), rtol=1e-9)
    # G_k = X_k X_k^T is the best rank-k approximation (Eckart-Young)
    Gk = res["coords"] @ res["coords"].T
    err = np.linalg.norm(res["G"] - Gk, "fro") ** 2
    assert np.isclose(err, (res["eigvals_all"][3:] ** 2).sum(), rtol=1e-8)


def test_sign_normalisation():
    X = np.array([[1.0, -3.0], [-2.0, 1.0], [2.0, 3.0]])
    Y = O.normalise_column_signs(X)
    assert np.array_equal(Y[:, 0], -X[:, 0])  # |-2| is the first maximum, made positive
    assert np.array_equal(Y[:, 1], -X[:, 1])  # first maximum is -3 at row 0


def test_randomized_exact_when_rank_at_most_l():
    X, _ = W.gaussian_mixture(250, 5, 3, 9.0, seed=1)
    D = W.euclidean_distances(X)
    full = O.full_mds(D, 4)
    rnd = O.rand_mds(D, 4, 3, 0, seed=7)  # l = 7 >= rank 5
    assert np.allclose(rnd["eigvals"], full["eigvals"], rtol=1e-11)
    assert np.allclose(rnd["coords"], full["coords"], rtol=0, atol=1e-8 * np.abs(full["coords"]).max())


def test_randomized_interlacing_and_convergence_in_q():
    reads, _ = W.amplicon_reads(400, 12, seed=2)
    D = W.hamming_distances(reads)
    full = O.full_mds(D, 8)
    lam = full["eigvals_all"]
    errs = []
    for q in range(5):
        rnd = O.rand_mds(D, 8, 4, q, seed=3, G=full["G"])
        th = rnd["theta"]
        # Cauchy interlacing for a compression Q^T G Q
        assert np.all(th <= lam[: th.size] + 1e-10 * lam[0])
        errs.append(np.max(np.abs(rnd["eigvals"] - lam[:8]) / lam[:8]))
    assert errs[-1] < 1e-6
    assert all(errs[i + 1] <= errs[i] * 1.05 + 1e-14 for i in range(4))


@pytest.mark.parametrize("q", [0, 1, 2])
def test_number_of_applications_of_G(q):
    # flat spectrum in [1, 2]: G^(2q+1) Omega is well conditioned, and spans
    # for different exponents are distinguishable
    rng = np.random.default_rng(q)
    n, k, p = 60, 3, 2
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.linspace(2.0, 1.0, n)
    G = (U * lam) @ U.T
    G = 0.5 * (G + G.T)
    rnd = O.rand_mds(np.zeros((n, n)), k, p, q, seed=4, G=G, keep_history=True)
    Q = rnd["Q"]
    Z = rnd["omega"]
    for _ in range(2 * q + 1):
        Z = G @ Z
    Qz = np.linalg.qr(Z)[0]
    s = np.linalg.svd(Q.T @ Qz, compute_uv=False)
    assert np.min(s) > 1 - 1e-10
    # one more application gives a clearly different span
    Qz2 = np.linalg.qr(G @ G @ Z)[0]
    assert np.min(np.linalg.svd(Q.T @ Qz2, compute_uv=False)) < 1 - 1e-6


def test_rayleigh_ritz_residuals_and_coordinates():
    reads, _ = W.amplicon_reads(300, 10, seed=5)
    D = W.hamming_distances(reads)
    rnd = O.rand_mds(D, 6, 6, 1, seed=1)
    Q, B = rnd["Q"], rnd["B"]
    assert np.max(np.abs(Q.T @ Q - np.eye(Q.shape[1]))) < 1e-13
    th, V = np.linalg.eigh(B)
    assert np.allclose(np.sort(th)[::-1], rnd["theta"], rtol=0, atol=1e-12 * abs(th).max())
    G = O.gram_matrix(D)
    U = rnd["coords"] / np.sqrt(rnd["eigvals"])[None, :]
    assert np.max(np.abs(U.T @ U - np.eye(6))) < 1e-12
    # Ritz values are Rayleigh quotients of the returned vectors
    assert np.allclose(np.einsum("ia,ij,ja->a", U, G, U), rnd["eigvals"], rtol=1e-12)


def test_non_euclidean_input_keeps_signs():
    reads, _ = W.amplicon_reads(300, 20, seed=6)
    D = W.hamming_distances(reads)
    full = O.full_mds(D, 5)
    assert np.min(full["eigvals_all"]) < -1e-6 * full["eigvals_all"][0]  # Sec. 6.3: not embeddable
    rnd = O.rand_mds(D, 5, 45, 2, seed=0)
    assert rnd["n_negative"] > 0
    assert np.all(rnd["coords"][:, rnd["eigvals"] <= 0] == 0)


def test_argument_validation():
    D = np.zeros((5, 5))
    with pytest.raises(ValueError):
        O.rand_mds(D, 4, 2, 0, 0)
    with pytest.raises(ValueError):
        O.rand_mds(D, 0, 2, 0, 0)


def test_forms_reduce_to_plain_on_representable_data():
    # A rank-2 cloud with l >= rank: the range is exact whatever the rounding
    # of X, so each form equals exact MDS up to the roundings of G and of Q in
    # the projection: fp32 operands move the eigenvalues by a few 2^-24, the
    # 16-bit projection of the bf16 form by up to 2^-15 (two-term operands
    # within 2^-17 each, a1 b1 dropped), its fp32 variant like fp32.
    X = np.array([[0, 0], [1, 0], [0, 1], [1, 1], [2, 0], [0, 2], [2, 2], [1, 2]], dtype=np.float64)
    D = np.sqrt(((X[:, None] - X[None]) ** 2).sum(-1))
    full = O.full_mds(D, 2)
    for form, tol in (("fp64", 1e-12), ("fp32", 1e-6), ("bf16_p32", 1e-6), ("bf16", 2.0 ** -15)):
        rnd = O.rand_mds(D, 2, 2, 1, seed=0, form=form)
        assert np.allclose(rnd["eigvals"], full["eigvals"], rtol=tol)


def test_bf16_form_perturbs_like_its_storage():
    reads, _ = W.amplicon_reads(600, 30, seed=7)
    D = W.hamming_distances(reads)
    a = O.rand_mds(D, 20, 10, 1, 0)["eigvals"]
    b = O.rand_mds(D, 20, 10, 1, 0, form="bf16_all")["eigvals"]
    c = O.rand_mds(D, 20, 10, 1, 0, form="fp32")["eigvals"]
    d = O.rand_mds(D, 20, 10, 1, 0, form="bf16")["eigvals"]
    e = O.rand_mds(D, 20, 10, 1, 0, form="bf16_p32")["eigvals"]
    eb, ec, ed, ee = (np.max(np.abs(v - a) / a) for v in (b, c, d, e))
    # every range pass on bf16 G: well above fp32; with 16-bit end passes and
    # an fp32 projection: far below; the 16-bit projection adds at most its
    # per-product bound 2^-15
    assert 1e-9 < ec < 1e-5 and ec < eb < 2e-2 and ee < eb / 10 and ed < 2.0 ** -15


def test_low_precision_schedule_has_16_bit_end_passes():
    # The bf16/fp8 forms take their first and last range application with G
    # to 16 bits (two-term bfloat16 expansion), X to 16 bits in the sketch of
    # Omega and bf16 in the last one: with q = 0 that single application is
    # the sketch and the whole range finder, so both forms are the same
    # method and stay within the 16-bit operand precision of the fp32 form;
    # with q >= 1 the bf16 form differs from the variant that runs every
    # application on the stored bf16 G.
    reads, _ = W.amplicon_reads(500, 20, seed=3)
    D = W.hamming_distances(reads)
    f32 = O.rand_mds(D, 8, 4, 0, 1, form="fp32")["eigvals"]
    b16 = O.rand_mds(D, 8, 4, 0, 1, form="bf16")["eigvals"]
    assert np.array_equal(O.rand_mds(D, 8, 4, 0, 1, form="fp8")["eigvals"], b16)
    assert 0 < np.max(np.abs(b16 - f32) / f32) < 1e-5
    assert [O.pass_dtypes("bf16", it, 2) for it in range(5)] == [
        ("bf16x2", "bf16x2"), ("bf16", "bf16"), ("bf16", "bf16"), ("bf16", "bf16"), ("bf16x2", "bf16")]
    assert O.pass_dtypes("bf16", 0, 0) == ("bf16x2", "bf16x2")
    assert all(O.pass_dtypes("bf16_all", it, 2) == ("bf16", "bf16") for it in range(5))
    a = O.rand_mds(D, 8, 4, 1, 1, form="bf16")["eigvals"]
    b = O.rand_mds(D, 8, 4, 1, 1, form="bf16_all")["eigvals"]
    assert not np.array_equal(a, b)


def test_two_term_bfloat16_rounding():
    # b0 + b1 with b0 = bf16(f), b1 = bf16(f - b0): against torch's own
    # float32 -> bfloat16 conversion (independent), the 2^-17 relative bound
    # of two nearest-even 8-bit roundings, and exact cases
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    x = rng.standard_normal(200000) * 10.0 ** rng.integers(-6, 6, 200000)
    got = O.round_to(x, "bf16x2")
    f = torch.from_numpy(x.astype(np.float32))
    b0 = f.to(torch.bfloat16).to(torch.float32)
    b1 = (f - b0).to(torch.bfloat16).to(torch.float32)
    assert np.array_equal(got, b0.double().numpy() + b1.double().numpy())
    f64 = x.astype(np.float32).astype(np.float64)
    assert np.all(np.abs(got - f64) <= 2.0 ** -17 * np.abs(f64))
    exact = np.array([1.0, 1.0 + 2.0 ** -12, -3.5, 0.0])  # at most 16 significant bits
    assert np.array_equal(O.round_to(exact, "bf16x2"), exact)


def test_fp32_end_passes_keep_bf16_within_1e3_near_degenerate():
    # 10-component mixture in 50 dims, k = 10: the k-th eigenvalue lies in the
    # noise bulk, where a sketch made only of bf16 applications moves the
    # Ritz values by more than 1e-3 relative to the fp64 method; with the two
    # end applications in fp32 the bf16 form stays well inside 1e-3.
    X, _ = W.gaussian_mixture(2000, 50, 10, 25.0, seed=0)
    D = W.euclidean_distances(X)
    ref = O.rand_mds(D, 10, 10, 1, 0)["eigvals"]
    err = {f: np.max(np.abs(O.rand_mds(D, 10, 10, 1, 0, form=f)["eigvals"] - ref) / np.abs(ref))
           for f in ("bf16", "bf16_all")}
    assert err["bf16"] < 2e-4 < 1e-3 < err["bf16_all"]
