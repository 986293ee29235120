"""CPU checks of two exact-arithmetic facts the HIP kernels rely on.

1. Three-term bf16 split of an fp32 value (the split fp32 G-passes):
   a0 = bf16(a), a1 = bf16(a - a0), a2 = bf16((a - a0) - a1), each rounded to
   nearest even, with both differences exact in fp32.  Then a0 + a1 + a2 == a
   exactly, and the six products a_p b_q with p + q <= 2 leave out less than
   2^-22 |a b|.
2. FP8 block quantisation: fl32(g / s) == fl32(g * (1 / s)) when the product
   and the reciprocal are formed in fp64 (an fp32 quotient is never an fp32
   midpoint and stays ~2^-48 away from one; the fp64 path errs by ~2^-52).

Both are checked on random and adversarial inputs with numpy, independently of
the kernels (bf16 rounding here is written on the bit pattern).
"""
import numpy as np


def bf16_rne(x):
    """fp32 -> bf16 (round to nearest even) -> fp32, on the bit pattern."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32)


def split3(a):
    a = np.asarray(a, dtype=np.float32)
    a0 = bf16_rne(a)
    r1 = (a - a0).astype(np.float32)
    a1 = bf16_rne(r1)
    r2 = (r1 - a1).astype(np.float32)
    a2 = bf16_rne(r2)
    return a0, a1, a2, r1, r2


def random_fp32(rng, n, lo=-40, hi=40):
    m = rng.uniform(1.0, 2.0, n)
    e = rng.integers(lo, hi, n)
    s = rng.choice([-1.0, 1.0], n)
    return (s * np.ldexp(m, e)).astype(np.float32)


def test_split3_is_exact():
    rng = np.random.default_rng(0)
    a = random_fp32(rng, 2_000_000)
    # adversarial: values whose low 16 bits sit on bf16 rounding ties
    u = a.view(np.uint32)
    ties = ((u & 0xFFFF0000) | 0x8000).view(np.float32)
    for x in (a, ties):
        a0, a1, a2, r1, r2 = split3(x)
        # both differences exact in fp32
        assert np.array_equal(r1.astype(np.float64), x.astype(np.float64) - a0.astype(np.float64))
        assert np.array_equal(r2.astype(np.float64), r1.astype(np.float64) - a1.astype(np.float64))
        # the last term needs no rounding: a0 + a1 + a2 == a exactly
        assert np.array_equal(a2, r2)
        total = a0.astype(np.float64) + a1.astype(np.float64) + a2.astype(np.float64)
        assert np.array_equal(total, x.astype(np.float64))
        ax = np.abs(x.astype(np.float64))
        assert np.all(np.abs(a1.astype(np.float64)) <= 2.0 ** -8 * ax * (1 + 2.0 ** -8))
        assert np.all(np.abs(a2.astype(np.float64)) <= 2.0 ** -16 * ax * (1 + 2.0 ** -7))


def test_six_products_bound():
    rng = np.random.default_rng(1)
    a = random_fp32(rng, 1_000_000, -20, 20)
    b = random_fp32(rng, 1_000_000, -20, 20)
    A = [t.astype(np.float64) for t in split3(a)[:3]]
    B = [t.astype(np.float64) for t in split3(b)[:3]]
    kept = sum(A[p] * B[q] for p in range(3) for q in range(3) if p + q <= 2)
    exact = a.astype(np.float64) * b.astype(np.float64)
    # the three dropped terms (products of terms below 2^-8 and 2^-16) are
    # below 2^-22 |a b|; the fp64 sums here are exact to far below that
    assert np.all(np.abs(exact - kept) <= 2.0 ** -22 * np.abs(exact))


def test_fp64_reciprocal_division_rounds_like_fp32_division():
    rng = np.random.default_rng(2)
    n = 3_000_000
    g = random_fp32(rng, n, -30, 10)
    # block scales as the quantiser forms them: s = fl32(max / 448)
    mx = np.abs(random_fp32(rng, n, -20, 10))
    s = (mx / np.float32(448.0)).astype(np.float32)
    want = (g / s).astype(np.float32)  # IEEE fp32 division, correctly rounded
    got = (g.astype(np.float64) * (1.0 / s.astype(np.float64))).astype(np.float32)
    assert np.array_equal(got, want)
    # near-midpoint quotients: g = s * m with m an fp32 midpoint, rounded to fp32
    m = random_fp32(rng, n, -5, 8).astype(np.float64)
    m = m * (1 + 2.0 ** -24)  # halfway towards the next fp32 value (roughly)
    s2 = np.abs(random_fp32(rng, n, -10, 5))
    g2 = (m * s2.astype(np.float64)).astype(np.float32)
    want2 = (g2 / s2).astype(np.float32)
    got2 = (g2.astype(np.float64) * (1.0 / s2.astype(np.float64))).astype(np.float32)
    assert np.array_equal(got2, want2)
