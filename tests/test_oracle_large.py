"""The row-blocked oracle equals the monolithic one (pin of the blocking)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytest.importorskip("torch")
from oracle import mds_oracle_large as OL  # noqa: E402


@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16"])
def test_blocked_matches_monolithic(form):
    reads, _ = W.amplicon_reads(700, 25, seed=4)
    D = W.hamming_distances(reads)
    a = O.rand_mds(D, 12, 8, 2, seed=3, form=form)
    b = OL.rand_mds_blocked(D, 12, 8, 2, seed=3, form=form, block=97)
    assert np.allclose(a["eigvals"], b["eigvals"], rtol=1e-12, atol=0)
    assert np.allclose(a["coords"], b["coords"], rtol=0, atol=1e-9 * np.abs(a["coords"]).max())


def test_blocked_stats():
    rng = np.random.default_rng(1)
    D = rng.random((301, 301)).astype(np.float32)
    r, c, m = O.centring_stats(D)
    rb, cb, mb = OL.centring_stats_blocked(D, block=64)
    assert np.allclose(r, rb, rtol=1e-14) and np.allclose(c, cb, rtol=1e-14)
    assert np.isclose(m, mb, rtol=1e-14)
    G = O.gram_matrix(D)
    X = rng.standard_normal((301, 5))
    assert np.allclose(OL.gram_apply_blocked(D, (r, c, m), X, block=50), G @ X, rtol=1e-12, atol=1e-12)
