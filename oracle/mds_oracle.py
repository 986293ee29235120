"""Plain float64 CPU oracle for dense random-projection classical MDS.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  The GPU library never calls it,
shares no code with it, and must fail loudly when its HIP extension is
missing rather than fall back to anything here.

What is computed (Blanchard et al., "A geometric view of Biodiversity:
scaling to metagenomics", Inria RR-9144):

* Gram matrix from distances -- Sec. 6.2, step 1 (the double-centring
  equation): gamma_ij = -1/2 (d_ij^2 - (1/n) sum_i d_ij^2
  - (1/n) sum_j d_ij^2 + (1/n^2) sum_ij d_ij^2).
* Exact classical MDS -- Sec. 6.2, steps 2 and 3: eigenpairs of G, X = U
  Lambda^{1/2}, keep the first k columns (``full_mds``).
* Random-projection MDS -- Sec. 3.2 and 3.3: an approximate rank-k spectral
  decomposition of G through the randomized range finder of Halko, Martinsson
  and Tropp (SIAM Review 2011), with power iterations and oversampling, then
  Rayleigh-Ritz on the small projected matrix (``rand_mds``).  The paper does
  not print the algorithm; the readings taken here are:
    - Gaussian test matrix Omega (n x l, l = k + p) from Philox4x64-10 and
      Box-Muller (``omega``);
    - q power iterations = q applications of G^T G = G^2, with an
      orthonormalisation after every application of G, so 2q + 1 range
      applications plus one projection application;
    - eigenpairs of the symmetric B = Q^T G Q keep their signs (G need not be
      positive semi-definite, Sec. 6.3); order is algebraic, descending;
      coordinates use sqrt(max(theta, 0));
    - each coordinate column is sign-normalised so that its entry of largest
      magnitude (lowest row index on ties) is positive.

Parity pins (tests/test_oracle_*.py): Euclidean point clouds (G equals the
centred Gram matrix of the points; eigenvalues equal squared singular values
of the centred cloud; the embedding reproduces D), row sums of G vanish,
trace identity, rank(G) <= l makes the randomized result exact, Cauchy
interlacing, monotone convergence in q, power count against an explicit
G^(2q+1) Omega, Philox known-answer vectors and numpy's independent Philox.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "philox4x64_10",
    "omega_words",
    "omega",
    "centring_stats",
    "gram_matrix",
    "gram_entries",
    "full_mds",
    "rand_mds",
    "orthonormal_basis",
    "normalise_column_signs",
    "round_to",
    "round_form",
    "e4m3_value",
    "fp8_block_quantize",
    "fp8_operand",
    "E4M3_MAX",
    "FP8_BLOCK",
    "FORMS",
]

# ---------------------------------------------------------------------------
# Philox4x64-10 counter-based generator
# (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3",
#  SC'11).  One block maps a 256-bit counter and a 128-bit key to 256 bits.
# ---------------------------------------------------------------------------
_M0 = np.uint64(0xD2E7470EE14C6C93)
_M1 = np.uint64(0xCA5A826395121157)
_W0 = 0x9E3779B97F4A7C15
_W1 = 0xBB67AE8584CAA73B
_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(m: np.uint64, x: np.ndarray):
    """(high, low) 64-bit halves of the 128-bit product m * x."""
    lo = m * x  # wraps modulo 2^64
    m0 = m & _MASK32
    m1 = m >> _S32
    x0 = x & _MASK32
    x1 = x >> _S32
    p00 = m0 * x0
    p01 = m0 * x1
    p10 = m1 * x0
    p11 = m1 * x1
    mid = (p00 >> _S32) + (p01 & _MASK32) + (p10 & _MASK32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64_10(ctr, key):
    """Philox4x64 with 10 rounds.

    ctr: uint64 array (..., 4); key: (k0, k1) integers.  Returns uint64
    array (..., 4).  Each round multiplies words 0 and 2 by the two round
    multipliers, swaps the halves and xors in the key; the key is bumped by
    the two Weyl constants between rounds.
    """
    c = np.array(ctr, dtype=np.uint64, copy=True)
    x0, x1, x2, x3 = (c[..., i].copy() for i in range(4))
    k0 = int(key[0]) & 0xFFFFFFFFFFFFFFFF
    k1 = int(key[1]) & 0xFFFFFFFFFFFFFFFF
    with np.errstate(over="ignore"):
        for rnd in range(10):
            if rnd > 0:
                k0 = (k0 + _W0) & 0xFFFFFFFFFFFFFFFF
                k1 = (k1 + _W1) & 0xFFFFFFFFFFFFFFFF
            hi0, lo0 = _mulhilo(_M0, x0)
            hi1, lo1 = _mulhilo(_M1, x2)
            x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(k0), lo1,
                              hi0 ^ x3 ^ np.uint64(k1), lo0)
    return np.stack([x0, x1, x2, x3], axis=-1)


def omega_words(seed: int, rows, blocks):
    """Raw Philox words for rows i and column blocks b (columns 4b..4b+3):
    block Philox4x64-10(counter = (i, b, 0, 0), key = (seed, 0))."""
    rows = np.asarray(rows, dtype=np.uint64)
    blocks = np.asarray(blocks, dtype=np.uint64)
    rows, blocks = np.broadcast_arrays(rows, blocks)
    ctr = np.zeros(rows.shape + (4,), dtype=np.uint64)
    ctr[..., 0] = rows
    ctr[..., 1] = blocks
    return philox4x64_10(ctr, (seed, 0))


_TWO_PI = 2.0 * math.pi
_TWO_M53 = 2.0 ** -53


def _box_muller(wa: np.ndarray, wb: np.ndarray):
    """Two standard normals from two 64-bit words (Box and Muller, 1958):
    u = (top 53 bits of wa + 1/2) 2^-53 in (0,1), v = (top 53 bits of wb)
    2^-53 in [0,1); z = sqrt(-2 ln u) (cos 2 pi v, sin 2 pi v)."""
    u = ((wa >> np.uint64(11)).astype(np.float64) + 0.5) * _TWO_M53
    v = (wb >> np.uint64(11)).astype(np.float64) * _TWO_M53
    rho = np.sqrt(-2.0 * np.log(u))
    ang = _TWO_PI * v
    return rho * np.cos(ang), rho * np.sin(ang)


def omega(seed: int, n: int, l: int, rows=None) -> np.ndarray:
    """Gaussian test matrix Omega (n x l float64), the random input of the
    range finder (Sec. 3.2, following Halko et al.).  Entry (i, j) depends
    only on (seed, i, j): words w0..w3 of block (i, j // 4) give
    (z0, z1) from (w0, w1) and (z2, z3) from (w2, w3); column 4b + t takes z_t.
    ``rows`` optionally selects a subset of rows (for sampled checks)."""
    rows = np.arange(n, dtype=np.uint64) if rows is None else np.asarray(rows, dtype=np.uint64)
    nb = (l + 3) // 4
    w = omega_words(seed, rows[:, None], np.arange(nb, dtype=np.uint64)[None, :])
    z0, z1 = _box_muller(w[..., 0], w[..., 1])
    z2, z3 = _box_muller(w[..., 2], w[..., 3])
    out = np.stack([z0, z1, z2, z3], axis=-1).reshape(len(rows), 4 * nb)
    return np.ascontiguousarray(out[:, :l])


# ---------------------------------------------------------------------------
# Double centring (Sec. 6.2, step 1)
# ---------------------------------------------------------------------------

def centring_stats(D):
    """Means of squared distances appearing in the Gram equation of Sec. 6.2:
    r_i = (1/n) sum_j d_ij^2 (row means), c_j = (1/n) sum_i d_ij^2 (column
    means), m = (1/n^2) sum_ij d_ij^2.  Squares are taken in float64 (exact
    for float32 inputs)."""
    D2 = np.asarray(D, dtype=np.float64) ** 2
    n = D2.shape[0]
    r = D2.sum(axis=1) / n
    c = D2.sum(axis=0) / n
    m = D2.sum() / (n * n)
    return r, c, m


def gram_matrix(D, stats=None) -> np.ndarray:
    """G = [gamma_ij] with gamma_ij = -1/2 (d_ij^2 - c_j - r_i + m), written in
    the order of the equation of Sec. 6.2, step 1."""
    D2 = np.asarray(D, dtype=np.float64) ** 2
    r, c, m = centring_stats(D) if stats is None else stats
    return -0.5 * (D2 - c[None, :] - r[:, None] + m)


def gram_entries(d_vals, r_i, c_j, m):
    """gamma_ij for sampled entries, given d_ij, r_i, c_j and m (same
    equation as ``gram_matrix``, one entry at a time)."""
    d2 = np.asarray(d_vals, dtype=np.float64) ** 2
    return -0.5 * (d2 - c_j - r_i + m)


# ---------------------------------------------------------------------------
# Storage roundings of the arithmetic forms
# ---------------------------------------------------------------------------

def round_to(x, dtype: str) -> np.ndarray:
    """Round float64 values to the storage type of a form and return them as
    float64: 'f64' keeps them, 'f32' rounds to nearest even, 'bf16' rounds to
    float32 and then to bfloat16 (8 significant bits), both nearest even."""
    x = np.asarray(x, dtype=np.float64)
    if dtype == "f64":
        return x.copy()
    f = x.astype(np.float32)
    if dtype == "f32":
        return f.astype(np.float64)
    if dtype != "bf16":
        raise ValueError(dtype)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)).astype(np.uint32)
    return (r << np.uint32(16)).view(np.float32).astype(np.float64)


E4M3_MAX = 448.0  # largest finite OCP FP8 E4M3 value (1.75 * 2^8)
FP8_BLOCK = 256   # side of the square blocks that share one scale


def e4m3_value(x) -> np.ndarray:
    """Value of the OCP FP8 E4M3 number nearest to each float (ties to even
    significand), saturating at +-448.  E4M3: 1 sign bit, 4 exponent bits
    with bias 7, 3 fraction bits; normal numbers (1 + f/8) 2^(e-7) for
    e = 1..15 (448 = 1.75 * 2^8 is the largest, the all-ones code is NaN),
    subnormals (f/8) 2^-6, i.e. multiples of 2^-9 below 2^-6."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    out = np.zeros_like(a)
    normal = a >= 2.0 ** -6
    f, E = np.frexp(a[normal])  # a = f 2^E, f in [0.5, 1)
    e = E - 1                    # a = (2 f) 2^e, 2 f in [1, 2)
    out[normal] = np.rint(2.0 * f * 8.0) / 8.0 * np.ldexp(1.0, e)  # np.rint: half to even
    out[~normal] = np.rint(a[~normal] * 2.0 ** 9) * 2.0 ** -9
    out = np.minimum(out, E4M3_MAX)
    return np.copysign(out, x)


def fp8_block_quantize(G: np.ndarray, block: int = FP8_BLOCK):
    """Per-block scaled FP8 storage of G: entries rounded to float32 g; for
    each block x block tile a float32 scale s = max|g| / 448 (1 for an
    all-zero tile); stored codes q = e4m3(fl32(g / s)).  Returns (q values,
    scale per entry), both float64 arrays of G's shape."""
    g = np.asarray(G, dtype=np.float64).astype(np.float32)
    n0, n1 = g.shape
    q = np.zeros(g.shape, dtype=np.float64)
    sc = np.ones(g.shape, dtype=np.float64)
    for i0 in range(0, n0, block):
        for j0 in range(0, n1, block):
            t = g[i0:i0 + block, j0:j0 + block]
            mx = np.float32(np.max(np.abs(t))) if t.size else np.float32(0.0)
            s = np.float32(mx / np.float32(E4M3_MAX)) if mx > 0 else np.float32(1.0)
            q[i0:i0 + block, j0:j0 + block] = e4m3_value((t / s).astype(np.float32))
            sc[i0:i0 + block, j0:j0 + block] = s
    return q, sc


def fp8_operand(G: np.ndarray) -> np.ndarray:
    """The G entries the FP8 form multiplies with: each stored code times its
    block scale in float32, rounded to bfloat16 (the MFMA operand type)."""
    q, sc = fp8_block_quantize(G)
    return round_to((q.astype(np.float32) * sc.astype(np.float32)).astype(np.float64), "bf16")


# Dtype of (G, X) in the range passes and in the projection pass of each form.
FORMS = {
    "fp64": {"range": ("f64", "f64"), "proj": ("f64", "f64")},
    "fp32": {"range": ("f32", "f32"), "proj": ("f32", "f32")},
    "bf16": {"range": ("bf16", "bf16"), "proj": ("f32", "f32")},
    "fp8": {"range": ("fp8blk", "bf16"), "proj": ("f32", "f32")},
}


def round_form(x, dtype: str) -> np.ndarray:
    """round_to, plus 'fp8blk': the block-scaled FP8 operand of a matrix."""
    return fp8_operand(x) if dtype == "fp8blk" else round_to(x, dtype)


# ---------------------------------------------------------------------------
# Helpers shared by both MDS variants of the oracle
# ---------------------------------------------------------------------------

def normalise_column_signs(X: np.ndarray) -> np.ndarray:
    """Flip each column so that its entry of largest magnitude is positive
    (lowest row index among exact ties).  Eigenvectors are defined only up to
    sign; this fixes one representative independently of the basis used."""
    X = np.array(X, copy=True)
    if X.shape[0] == 0:
        return X
    idx = np.argmax(np.abs(X), axis=0)  # first maximum = lowest index
    s = np.sign(X[idx, np.arange(X.shape[1])])
    s[s == 0] = 1.0
    return X * s[None, :]


def _sorted_eigh(A: np.ndarray):
    """Eigenpairs of a symmetric matrix in algebraic descending order
    (stable: ties keep the lower original index)."""
    w, V = np.linalg.eigh(A)
    order = np.argsort(-w, kind="stable")
    return w[order], V[:, order]


def orthonormal_basis(Y: np.ndarray) -> np.ndarray:
    """Orthonormal basis of range(Y) by Householder QR (LAPACK geqrf/orgqr).
    Only span(Q) matters to the method; the GPU library may use another
    orthonormaliser."""
    Q, _ = np.linalg.qr(Y, mode="reduced")
    return Q


# ---------------------------------------------------------------------------
# Exact classical MDS (Sec. 6.2, steps 1-3)
# ---------------------------------------------------------------------------

def full_mds(D, k: int):
    """Exact classical MDS through a full symmetric eigendecomposition of G.

    Returns dict with eigvals (top k, algebraic descending), all eigenvalues,
    coords X_k = U_k diag(sqrt(max(lambda, 0))) (sign-normalised), and G."""
    G = gram_matrix(D)
    lam, U = _sorted_eigh(G)
    X = U[:, :k] * np.sqrt(np.maximum(lam[:k], 0.0))[None, :]
    return {"eigvals": lam[:k].copy(), "eigvals_all": lam, "coords": normalise_column_signs(X),
            "G": G}


# ---------------------------------------------------------------------------
# Random-projection MDS (Sec. 3.2-3.3 with the Halko et al. range finder)
# ---------------------------------------------------------------------------

def rand_mds(D, k: int, p: int, q: int, seed: int, G=None, keep_history=False, form: str = "fp64"):
    """Randomized classical MDS.

    ``form`` names the storage precision of the operands of each product with
    G (see ``FORMS``): before every application Y = G X both G and X are
    rounded to that form's dtype and the product is then taken exactly in
    float64 arithmetic.  Everything else stays float64.  form="fp64" is the
    plain method.

    Steps, in order:
      1. G from D (Sec. 6.2, step 1).
      2. Omega = omega(seed, n, l), l = k + p.
      3. Y = G Omega; Q = orth(Y).
      4. q times: {Y = G Q; Q = orth(Y); Y = G Q; Q = orth(Y)} (G^T = G).
      5. Y = G Q; B = Q^T Y, symmetrised as (B + B^T)/2.
      6. eigenpairs (theta, V) of B, algebraic descending.
      7. eigvals = theta[:k]; X = Q V[:, :k] diag(sqrt(max(theta[:k], 0))),
         columns sign-normalised.
    """
    D = np.asarray(D)
    n = D.shape[0]
    l = k + p
    if not (1 <= k and p >= 0 and l <= n and q >= 0):
        raise ValueError("need 1 <= k, p >= 0, k + p <= n, q >= 0")
    if G is None:
        G = gram_matrix(D)
    gr, xr = FORMS[form]["range"]
    gp, xp = FORMS[form]["proj"]
    Gr = round_form(G, gr)
    Gp = round_form(G, gp)
    Om = omega(seed, n, l)
    history = []
    Y = Gr @ round_to(Om, xr)
    Q = orthonormal_basis(Y)
    if keep_history:
        history.append(Q.copy())
    for _ in range(q):
        for _half in range(2):
            Y = Gr @ round_to(Q, xr)
            Q = orthonormal_basis(Y)
            if keep_history:
                history.append(Q.copy())
    Y = Gp @ round_to(Q, xp)
    B = Q.T @ Y
    B = 0.5 * (B + B.T)
    theta, V = _sorted_eigh(B)
    X = Q @ V[:, :k] * np.sqrt(np.maximum(theta[:k], 0.0))[None, :]
    out = {
        "eigvals": theta[:k].copy(),
        "theta": theta,
        "coords": normalise_column_signs(X),
        "Q": Q,
        "B": B,
        "omega": Om,
        "frob2": float(np.sum(G * G)),
        "trace": float(np.trace(G)),
        "n_negative": int(np.sum(theta < -1e-12 * max(abs(theta[0]), 1e-300))),
    }
    if keep_history:
        out["history"] = history
    return out
