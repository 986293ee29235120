"""Pins of the oracle's FP8 form: the E4M3 rounding against PyTorch's own
float8_e4m3fn conversion (an independent implementation), the format's
closed-form facts, and the block scaling."""
import numpy as np
import pytest

import oracle as O
import workloads as W

torch = pytest.importorskip("torch")


def torch_e4m3(x):
    return torch.from_numpy(np.asarray(x, dtype=np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()


def test_e4m3_matches_torch_on_every_code_and_midpoint():
    codes = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    vals = np.unique(codes[np.isfinite(codes)])
    assert len(vals) == 253 and vals.max() == 448.0 and vals[vals > 0].min() == 2.0 ** -9
    assert np.array_equal(O.e4m3_value(vals), vals)  # representable values are fixed points
    mids = 0.5 * (vals[1:] + vals[:-1])  # exact ties: round half to even significand
    assert np.array_equal(O.e4m3_value(mids), torch_e4m3(mids))
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(-448, 448, 200000), rng.normal(0, 1e-2, 200000),
                        rng.normal(0, 1e-3, 50000)]).astype(np.float32)
    assert np.array_equal(O.e4m3_value(x), torch_e4m3(x))


def test_e4m3_closed_forms():
    assert O.e4m3_value(1.0 + 1.0 / 16) == 1.0      # tie -> even (1.000)
    assert O.e4m3_value(1.0 + 3.0 / 16) == 1.25     # tie -> even (1.010)
    assert O.e4m3_value(3.0 * 2 ** -10) == 2 ** -8  # subnormal tie 1.5 ulp -> 2 ulp
    assert O.e4m3_value(460.0) == 448.0 and O.e4m3_value(-1e6) == -448.0  # saturation
    x = np.linspace(2 ** -6, 448, 10001)
    assert np.max(np.abs(O.e4m3_value(x) - x) / x) <= 2.0 ** -4  # half a unit of the 3-bit fraction


def test_block_quantize_scales():
    rng = np.random.default_rng(1)
    G = rng.normal(0, 3.0, (600, 520))
    G[256:512, 0:256] = 0.0  # an all-zero block keeps scale 1
    q, sc = O.fp8_block_quantize(G)
    for i0 in range(0, 600, 256):
        for j0 in range(0, 520, 256):
            t = G[i0:i0 + 256, j0:j0 + 256].astype(np.float32)
            s = sc[i0, j0]
            assert np.all(sc[i0:i0 + 256, j0:j0 + 256] == s)
            if np.max(np.abs(t)) == 0:
                assert s == 1.0 and np.all(q[i0:i0 + 256, j0:j0 + 256] == 0)
            else:
                assert s == np.float32(np.float32(np.max(np.abs(t))) / np.float32(448.0))
                assert np.max(np.abs(q[i0:i0 + 256, j0:j0 + 256])) == 448.0
    A = O.fp8_operand(G)
    big = np.abs(G) > 1.0
    assert np.max(np.abs(A[big] - G[big]) / np.abs(G[big])) < 2.0 ** -4 + 2.0 ** -8


def test_fp8_form_runs_and_is_close():
    reads, _ = W.amplicon_reads(1500, 30, seed=2)
    D = W.hamming_distances(reads)
    ref = O.rand_mds(D, 20, 10, 2, 0)
    f8 = O.rand_mds(D, 20, 10, 2, 0, form="fp8")
    err = np.max(np.abs(f8["eigvals"] - ref["eigvals"]) / np.abs(ref["eigvals"]))
    assert err < 1e-2
