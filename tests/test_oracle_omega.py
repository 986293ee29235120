"""Pins for the oracle's test-matrix generator (Philox4x64-10 + Box-Muller).

The random test matrix is the Gaussian sketch of the range finder (Sec. 3.2).
Pinned against: the generator's published known-answer vectors, numpy's
independent Philox implementation, scalar libm evaluation of Box-Muller, and
distributional checks.
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


def _scalar_normals(w):
    out = []
    for a, b in ((w[0], w[1]), (w[2], w[3])):
        u = ((a >> 11) + 0.5) * 2.0 ** -53
        v = (b >> 11) * 2.0 ** -53
        rho = math.sqrt(-2.0 * math.log(u))
        out += [rho * math.cos(2.0 * math.pi * v), rho * math.sin(2.0 * math.pi * v)]
    return out


def test_box_muller_against_scalar_libm():
    seed, n, l = 5, 37, 13
    Om = O.omega(seed, n, l)
    for i in (0, 1, 17, 36):
        for b in range((l + 3) // 4):
            words = [int(x) for x in O.omega_words(seed, np.array([i]), np.array([b]))[0]]
            want = _scalar_normals(words)
            for t in range(4):
                j = 4 * b + t
                if j < l:
                    assert abs(Om[i, j] - want[t]) <= 4e-16 * max(1.0, abs(want[t]))


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
