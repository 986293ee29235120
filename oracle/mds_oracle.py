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

import numpy as np

__all__ = [
    "philox4x64_10",
    "omega_words",
    "omega",
    "ln_unit",
    "sincos_2pi",
    "centring_stats",
    "gram_matrix",
    "gram_entries",
    "full_mds",
    "jacobi_eigh",
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
    "pass_dtypes",
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


_TWO_M53 = 2.0 ** -53

# ---------------------------------------------------------------------------
# ln, sin and cos for Box-Muller, written from the mathematics with + - * /
# and sqrt only, in a fixed order (numpy float64 arrays: IEEE round to
# nearest, no fused multiply-add), so that the library's device code, which
# evaluates the same expressions in the same order, produces the same bits.
# ---------------------------------------------------------------------------
_LN2_HI = float.fromhex("0x1.62e42ff000000p-1")   # ln 2 rounded to a 32-bit fraction (e * _LN2_HI is exact)
_LN2_LO = float.fromhex("-0x1.718432a1b0e26p-35")  # ln 2 - _LN2_HI, rounded
_SQRT_HALF = float.fromhex("0x1.6a09e667f3bcdp-1")
_PI_4 = float.fromhex("0x1.921fb54442d18p-1")     # pi / 4, rounded
# 1 / (2j + 1) for j = 1..10: the odd terms of 2 atanh(s) = ln((1 + s) / (1 - s))
_ATANH = [float.fromhex(h) for h in (
    "0x1.5555555555555p-2", "0x1.999999999999ap-3", "0x1.2492492492492p-3", "0x1.c71c71c71c71cp-4",
    "0x1.745d1745d1746p-4", "0x1.3b13b13b13b14p-4", "0x1.1111111111111p-4", "0x1.e1e1e1e1e1e1ep-5",
    "0x1.af286bca1af28p-5", "0x1.8618618618618p-5")]
# (-1)^j / (2j + 1)! for j = 1..8 (sine) and (-1)^j / (2j)! for j = 1..9 (cosine)
_SIN = [float.fromhex(h) for h in (
    "-0x1.5555555555555p-3", "0x1.1111111111111p-7", "-0x1.a01a01a01a01ap-13", "0x1.71de3a556c734p-19",
    "-0x1.ae64567f544e4p-26", "0x1.6124613a86d09p-33", "-0x1.ae7f3e733b81fp-41", "0x1.952c77030ad4ap-49")]
_COS = [float.fromhex(h) for h in (
    "-0x1.0000000000000p-1", "0x1.5555555555555p-5", "-0x1.6c16c16c16c17p-10", "0x1.a01a01a01a01ap-16",
    "-0x1.27e4fb7789f5cp-22", "0x1.1eed8eff8d898p-29", "-0x1.93974a8c07c9dp-37", "0x1.ae7f3e733b81fp-45",
    "-0x1.6827863b97d97p-53")]


def ln_unit(u: np.ndarray) -> np.ndarray:
    """Natural logarithm of u in (0, 1].  u = m 2^e with m in [sqrt(1/2),
    sqrt(2)) (exact split); ln m = 2 atanh(s) with s = (m - 1) / (m + 1),
    |s| <= 0.172, summed as s + s z P(z), z = s^2, P the odd-term series to
    z^9 / 21 (remainder below 2^-54 relative); ln u = e ln2_hi + (e ln2_lo +
    ln m) with ln 2 split so that e ln2_hi is exact."""
    u = np.asarray(u, dtype=np.float64)
    f, e = np.frexp(u)  # u = f 2^e, f in [1/2, 1)
    low = f < _SQRT_HALF
    m = np.where(low, f + f, f)
    e = np.where(low, e - 1, e).astype(np.float64)
    s = (m - 1.0) / (m + 1.0)
    z = s * s
    p = np.full_like(s, _ATANH[-1])
    for c in reversed(_ATANH[:-1]):
        p = p * z + c
    t = s * (z * p)
    lnm = (s + t) * 2.0
    return e * _LN2_HI + (e * _LN2_LO + lnm)


def sincos_2pi(v: np.ndarray):
    """(sin 2 pi v, cos 2 pi v) for v in [0, 1).  Octant reduction of the
    dyadic v (exact): 8 v = o + f, x = a pi/4 with a = f (o even) or 1 - f
    (o odd), x in [0, pi/4]; Taylor series of sin and cos in z = x^2 to x^17
    and x^18 (remainders below 2^-55); the octant maps (sin x, cos x) to the
    angle by symmetry (exact sign changes and swaps)."""
    v = np.asarray(v, dtype=np.float64)
    t = v * 8.0
    o = np.floor(t)
    f = t - o
    odd = (o.astype(np.int64) & 1) == 1
    a = np.where(odd, 1.0 - f, f)
    x = a * _PI_4
    z = x * x
    ps = np.full_like(x, _SIN[-1])
    for c in reversed(_SIN[:-1]):
        ps = ps * z + c
    sx = x + (x * z) * ps
    pc = np.full_like(x, _COS[-1])
    for c in reversed(_COS[:-1]):
        pc = pc * z + c
    cx = 1.0 + z * pc
    oi = o.astype(np.int64)
    # octant o: angle = o pi/4 + f pi/4; sin / cos of it from (sx, cx)
    swap = (oi == 1) | (oi == 2) | (oi == 5) | (oi == 6)
    s_out = np.where(swap, cx, sx)
    c_out = np.where(swap, sx, cx)
    s_neg = oi >= 4
    c_neg = (oi >= 2) & (oi <= 5)
    return np.where(s_neg, -s_out, s_out), np.where(c_neg, -c_out, c_out)


def _box_muller(wa: np.ndarray, wb: np.ndarray):
    """Two standard normals from two 64-bit words (Box and Muller, 1958):
    u = (top 53 bits of wa + 1/2) 2^-53 in (0,1), v = (top 53 bits of wb)
    2^-53 in [0,1); z = sqrt(-2 ln u) (cos 2 pi v, sin 2 pi v), with the
    ln, sin and cos above."""
    u = ((wa >> np.uint64(11)).astype(np.float64) + 0.5) * _TWO_M53
    v = (wb >> np.uint64(11)).astype(np.float64) * _TWO_M53
    rho = np.sqrt(-2.0 * ln_unit(u))
    sn, cs = sincos_2pi(v)
    return rho * cs, rho * sn


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

def _bf16_of_f32(f: np.ndarray) -> np.ndarray:
    """float32 array -> nearest-even bfloat16 values, as float32."""
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)).astype(np.uint32)
    return (r << np.uint32(16)).view(np.float32)


def round_to(x, dtype: str) -> np.ndarray:
    """Round float64 values to the storage type of a form and return them as
    float64: 'f64' keeps them, 'f32' rounds to nearest even, 'bf16' rounds to
    float32 and then to bfloat16 (8 significant bits), both nearest even;
    'bf16x2' is the sum of the first two terms of the bfloat16 expansion of
    the float32 value f: b0 = bf16(f), b1 = bf16(f - b0) (f - b0 is exact in
    float32), about 16 significant bits."""
    x = np.asarray(x, dtype=np.float64)
    if dtype == "f64":
        return x.copy()
    f = x.astype(np.float32)
    if dtype == "f32":
        return f.astype(np.float64)
    if dtype == "bf16":
        return _bf16_of_f32(f).astype(np.float64)
    if dtype == "bf16x2":
        b0 = _bf16_of_f32(f)
        b1 = _bf16_of_f32((f - b0).astype(np.float32))
        return b0.astype(np.float64) + b1.astype(np.float64)
    raise ValueError(dtype)


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


# Dtype of (G, X) in the range passes and in the projection pass of each
# form.  The low-precision forms ("bf16", "fp8") run the first and the last
# range pass with G to about 16 significant bits (the two-term bfloat16
# expansion of its float32 value) and only the passes between them on the
# stored low-precision G (the sketch of Omega and the final basis then carry
# no bf16/fp8 rounding of G); "bf16_all" and "fp8_all" run every range pass
# on the stored G.  X takes 16 bits as well in the sketch of Omega and is
# rounded to bfloat16 in the last range pass.  Their projection (the
# "refinement" pass) takes both operands to 16 bits; "bf16_p32" and
# "fp8_p32" make it an fp32 pass.  "bf16_f32g" takes float32 in place of the
# two-term expansions (the batched kernel's arithmetic).
_F32 = ("f32", "f32")
_X2 = ("bf16x2", "bf16x2")  # 16-bit sketch of Omega and projection
_X1 = ("bf16x2", "bf16")    # last 16-bit range pass
FORMS = {
    "fp64": {"first": ("f64", "f64"), "range": ("f64", "f64"), "last": ("f64", "f64"), "proj": ("f64", "f64")},
    "fp32": {"first": _F32, "range": _F32, "last": _F32, "proj": _F32},
    "bf16": {"first": _X2, "range": ("bf16", "bf16"), "last": _X1, "proj": _X2},
    "fp8": {"first": _X2, "range": ("fp8blk", "bf16"), "last": _X1, "proj": _X2},
    "bf16_p32": {"first": _X2, "range": ("bf16", "bf16"), "last": _X1, "proj": _F32},
    "fp8_p32": {"first": _X2, "range": ("fp8blk", "bf16"), "last": _X1, "proj": _F32},
    "bf16_all": {"first": ("bf16", "bf16"), "range": ("bf16", "bf16"), "last": ("bf16", "bf16"), "proj": _X2},
    "fp8_all": {"first": ("fp8blk", "bf16"), "range": ("fp8blk", "bf16"), "last": ("fp8blk", "bf16"),
                "proj": _X2},
    "bf16_f32g": {"first": _F32, "range": ("bf16", "bf16"), "last": ("f32", "bf16"), "proj": _F32},
}


def pass_dtypes(form: str, it: int, q: int):
    """(G dtype, X dtype) of range application `it` (0-based, of 2q + 1)."""
    f = FORMS[form]
    return f["first"] if it == 0 else (f["last"] if it == 2 * q else f["range"])


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


def jacobi_eigh(A: np.ndarray, tol: float = 1e-15, max_sweeps: int = 60):
    """Eigenpairs of a symmetric matrix by the cyclic Jacobi method, for small
    matrices (pure Python loops over the pairs).

    Each sweep visits the pairs (p, q), p < q, row by row; for a nonzero
    a_pq the 2 x 2 symmetric Schur rotation J (c = 1 / sqrt(1 + t^2),
    s = t c, t the smaller root of t^2 + 2 tau t - 1 = 0 with
    tau = (a_qq - a_pp) / (2 a_pq)) zeroes a_pq in A <- J^T A J, and the
    rotations accumulate in V <- V J (Golub and Van Loan, Matrix
    Computations, the symmetric Schur decomposition and the cyclic Jacobi
    method).  Sweeps stop once the off-diagonal Frobenius norm is at most
    tol times the Frobenius norm of A.  Returns the eigenvalues in algebraic
    descending order (stable on ties) and the eigenvectors as columns."""
    A = np.array(A, dtype=np.float64, copy=True)
    n = A.shape[0]
    V = np.eye(n)
    scale = np.sqrt(np.sum(A * A))
    for _ in range(max_sweeps):
        off = np.sqrt(2.0 * np.sum(np.triu(A, 1) ** 2))  # summed directly: no cancellation
        if off <= tol * scale:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = A[p, q]
                if apq == 0.0:
                    continue
                tau = (A[q, q] - A[p, p]) / (2.0 * apq)
                t = (1.0 if tau >= 0.0 else -1.0) / (abs(tau) + np.sqrt(1.0 + tau * tau))
                c = 1.0 / np.sqrt(1.0 + t * t)
                s = t * c
                cp, cq = A[:, p].copy(), A[:, q].copy()  # A J
                A[:, p], A[:, q] = c * cp - s * cq, s * cp + c * cq
                rp, rq = A[p, :].copy(), A[q, :].copy()  # J^T (A J)
                A[p, :], A[q, :] = c * rp - s * rq, s * rp + c * rq
                vp, vq = V[:, p].copy(), V[:, q].copy()
                V[:, p], V[:, q] = c * vp - s * vq, s * vp + c * vq
    w = np.diag(A).copy()
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

def full_mds(D, k: int, method: str = "eigh"):
    """Exact classical MDS through a full symmetric eigendecomposition of G
    (LAPACK, or with method="jacobi" the cyclic Jacobi method of
    ``jacobi_eigh``, for small n).

    Returns dict with eigvals (top k, algebraic descending), all eigenvalues,
    coords X_k = U_k diag(sqrt(max(lambda, 0))) (sign-normalised), and G."""
    G = gram_matrix(D)
    if method == "jacobi":
        lam, U = jacobi_eigh(G)
    elif method == "eigh":
        lam, U = _sorted_eigh(G)
    else:
        raise ValueError(f"unknown method {method!r}")
    X = U[:, :k] * np.sqrt(np.maximum(lam[:k], 0.0))[None, :]
    return {"eigvals": lam[:k].copy(), "eigvals_all": lam, "coords": normalise_column_signs(X),
            "G": G}


# ---------------------------------------------------------------------------
# Random-projection MDS (Sec. 3.2-3.3 with the Halko et al. range finder)
# ---------------------------------------------------------------------------

def rand_mds(D, k: int, p: int, q: int, seed: int, G=None, keep_history=False, form: str = "fp64"):
    """Randomized classical MDS.

    ``form`` names the storage precision of the operands of each product with
    G (see ``FORMS`` and ``pass_dtypes``): before every application Y = G X
    both G and X are rounded to that pass's dtypes and the product is then
    taken exactly in float64 arithmetic.  Everything else stays float64.
    form="fp64" is the plain method.

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
    rounded = {}

    def g_as(dt):
        if dt not in rounded:
            rounded[dt] = round_form(G, dt)
        return rounded[dt]

    gp, xp = FORMS[form]["proj"]
    Om = omega(seed, n, l)
    history = []
    Q = Om
    for it in range(2 * q + 1):  # Omega, then q times two applications (G^T = G)
        gr, xr = pass_dtypes(form, it, q)
        Y = g_as(gr) @ round_to(Q, xr)
        Q = orthonormal_basis(Y)
        if keep_history:
            history.append(Q.copy())
    Y = g_as(gp) @ round_to(Q, xp)
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
