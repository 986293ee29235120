"""Pins for the oracle's test-matrix generator (Philox4x64-10 + Box-Muller).

The random test matrix is the Gaussian sketch of the range finder (Sec. 3.2).
Pinned against: the generator's published known-answer vectors, numpy's
independent Philox implementation, a long double evaluation of Box-Muller with
the C library's log, sin and cos (the project-defined ln, sin and cos within a
few ulps), and distributional checks.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O
from conftest import load_kat

M64 = (1 << 64) - 1


def test_philox_known_answers():
    for row in load_kat("philox4x64_10_kat.txt"):
        ctr, key, want = row[0:4], row[4:6], row[6:10]
        got = O.philox4x64_10(np.array(ctr, dtype=np.uint64), key)
        assert [int(x) for x in got] == want


def _numpy_block(ctr, key):
    """numpy's Philox increments its 256-bit counter before producing a block,
    so the block at counter c comes from a generator started at c - 1."""
    c = list(ctr)
    for w in range(4):  # subtract one with borrow, word 0 least significant
        if c[w] > 0:
            c[w] -= 1
            break
        c[w] = M64
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(c, dtype=np.uint64))
    return [int(x) for x in g.random_raw(4)]


def test_philox_matches_numpy_implementation():
    rng = np.random.default_rng(123)
    cases = [([0, 0, 0, 0], [0, 0]), ([0, 5, 0, 0], [7, 0]), ([1, 0, 0, 0], [2 ** 63, 0])]
    for _ in range(40):
        ctr = [int(x) for x in rng.integers(0, 2 ** 63, size=4, dtype=np.int64)]
        key = [int(x) for x in rng.integers(0, 2 ** 63, size=2, dtype=np.int64)]
        cases.append((ctr, key))
    for ctr, key in cases:
        got = [int(x) for x in O.philox4x64_10(np.array(ctr, dtype=np.uint64), key)]
        assert got == _numpy_block(ctr, key), (ctr, key)


def test_omega_words_use_row_and_block_counters():
    seed = 99
    w = O.omega_words(seed, np.array([[3]]), np.array([[2]]))[0, 0]
    assert [int(x) for x in w] == _numpy_block([3, 2, 0, 0], [seed, 0])


def _long_double_normals(w):
    """Box-Muller of one block evaluated in long double with the C library's
    log, sqrt, cos and sin (an independent evaluation at higher precision)."""
    two_pi = np.longdouble("6.283185307179586476925286766559005768")
    out = []
    for a, b in ((w[0], w[1]), (w[2], w[3])):
        u = np.longdouble((a >> 11)) + np.longdouble(0.5)
        u = u * np.longdouble(2.0 ** -53)
        v = np.longdouble(b >> 11) * np.longdouble(2.0 ** -53)
        rho = np.sqrt(np.longdouble(-2.0) * np.log(u))
        out += [rho * np.cos(two_pi * v), rho * np.sin(two_pi * v)]
    return out


def test_box_muller_against_long_double_libm():
    seed, n, l = 5, 37, 13
    Om = O.omega(seed, n, l)
    worst = 0.0
    for i in (0, 1, 17, 36):
        for b in range((l + 3) // 4):
            words = [int(x) for x in O.omega_words(seed, np.array([i]), np.array([b]))[0]]
            want = _long_double_normals(words)
            for t in range(4):
                j = 4 * b + t
                if j < l:
                    err = abs(np.longdouble(Om[i, j]) - want[t]) / max(np.longdouble(1.0), abs(want[t]))
                    worst = max(worst, float(err))
    assert worst <= 4 * 2.0 ** -53


def test_omega_entry_depends_only_on_seed_row_col():
    a = O.omega(11, 50, 21)
    b = O.omega(11, 80, 32)
    assert np.array_equal(a, b[:50, :21])
    rows = np.array([0, 7, 49])
    assert np.array_equal(O.omega(11, 50, 21, rows=rows), a[rows])
    assert not np.array_equal(a, O.omega(12, 50, 21))


def test_omega_is_standard_normal():
    z = O.omega(0, 20000, 16).ravel()
    assert abs(z.mean()) < 5.0 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5.0 * math.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # independence of the cos/sin pair and of neighbouring columns
    cc = np.corrcoef(O.omega(1, 20000, 8).T)
    assert np.max(np.abs(cc - np.eye(8))) < 5.0 / math.sqrt(20000)


def test_uniforms_open_interval():
    # extreme words: u must stay in (0,1) so log(u) is finite
    w = np.array([0, M64], dtype=np.uint64)
    z0, z1 = O.mds_oracle._box_muller(w, w[::-1].copy())
    assert np.all(np.isfinite(z0)) and np.all(np.isfinite(z1))


def test_round_to_bf16_and_f32():
    # ties to even at 8 significant bits
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -8 + 2.0 ** -20, -2.5e-3, 0.0])
    want = np.array([1.0, 1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7, None, 0.0], dtype=object)
    got = O.round_to(x, "bf16")
    for g, w in zip(got, want):
        if w is not None:
            assert g == w
    # against torch's independent float32 -> bfloat16 conversion
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    v = (rng.standard_normal(10000) * 10.0 ** rng.integers(-5, 5, 10000)).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(O.round_to(v.astype(np.float64), "bf16"), ref)
    assert np.array_equal(O.round_to(x, "f32"), x.astype(np.float32).astype(np.float64))
    assert np.array_equal(O.round_to(x, "f64"), x)


def _ulps(got, ref):
    """|got - ref| in units of the float64 spacing at ref (ref in long double)."""
    ref64 = ref.astype(np.float64)
    spacing = np.spacing(np.abs(ref64)).astype(np.longdouble)
    return np.abs(got.astype(np.longdouble) - ref) / spacing


def test_ln_unit_within_ulps_of_long_double_log():
    # the project-defined ln of Box-Muller against the C library's long double
    # log (an independent evaluation in 64-bit precision); every u the
    # generator can produce is ((w >> 11) + 1/2) 2^-53
    rng = np.random.default_rng(3)
    k = rng.integers(0, 2 ** 53, 200000, dtype=np.int64)
    k = np.concatenate([k, [0, 1, 2, 2 ** 52 - 1, 2 ** 52, 2 ** 53 - 1, 6369051672525772, 6369051672525773]])
    u = (k.astype(np.float64) + 0.5) * 2.0 ** -53
    got = O.ln_unit(u)
    ref = np.log(u.astype(np.longdouble))
    assert np.max(_ulps(got, ref)) <= 2.0
    assert O.ln_unit(np.array([1.0]))[0] == 0.0
    assert O.ln_unit(np.array([0.5]))[0] == -float.fromhex("0x1.62e42fefa39efp-1")  # -ln 2 rounded


def test_sincos_2pi_within_ulps_of_long_double():
    rng = np.random.default_rng(4)
    k = rng.integers(0, 2 ** 53, 200000, dtype=np.int64)
    k = np.concatenate([k, np.arange(0, 2 ** 53, 2 ** 50), np.arange(0, 2 ** 53, 2 ** 50) + 1,
                        np.arange(2 ** 50, 2 ** 53 + 1, 2 ** 50) - 1])
    v = k.astype(np.float64) * 2.0 ** -53
    sn, cs = O.sincos_2pi(v)
    two_pi = np.longdouble("6.283185307179586476925286766559005768")
    ang = v.astype(np.longdouble) * two_pi
    # absolute error in units of 2^-53 (the result spacing near 1): sin and
    # cos both lose relative accuracy where they pass through zero
    for got, ref in ((sn, np.sin(ang)), (cs, np.cos(ang))):
        err = np.abs(got.astype(np.longdouble) - ref) / np.longdouble(2.0 ** -53)
        assert np.max(err) <= 4.0
        assert np.all(np.abs(got) <= 1.0)
    # octant points: exact zeros and ones
    q = np.array([0.0, 0.25, 0.5, 0.75])
    sq, cq = O.sincos_2pi(q)
    assert np.array_equal(np.abs(sq), [0.0, 1.0, 0.0, 1.0]) and np.array_equal(np.abs(cq), [1.0, 0.0, 1.0, 0.0])
    assert np.array_equal(np.sign(sq[[1, 3]]), [1.0, -1.0]) and np.array_equal(np.sign(cq[[0, 2]]), [1.0, -1.0])
    # sin^2 + cos^2 = 1 to rounding
    assert np.max(np.abs(sn * sn + cs * cs - 1.0)) < 8e-16
