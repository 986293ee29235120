"""GPU input generators reproduce the numpy recipes (input generation only)."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from workloads import gpu as WG  # noqa: E402


@pytest.mark.parametrize("n,refs,length", [(3001, 40, 400), (700, 5, 130)])
def test_hamming_generator_bit_exact(n, refs, length):
    print(f"[gen] hamming n={n} L={length}", flush=True)
    reads, _ = W.amplicon_reads(n, refs, seed=3, length=length)
    got = WG.hamming_from_reads(reads).cpu().numpy()
    assert np.array_equal(got, W.hamming_distances(reads))


def test_euclid_generator():
    print("[gen] euclid n=1500 dim=50", flush=True)
    X, _ = W.gaussian_mixture(1500, 50, 10, 25.0, seed=0)
    ref64 = W.euclidean_distances(X)
    got64 = WG.euclidean_from_points(X, dtype="f64").cpu().numpy()
    assert np.max(np.abs(got64 - ref64) / np.maximum(ref64, 1e-300)) < 4e-16
    got32 = WG.euclidean_from_points(X, dtype="f32").cpu().numpy()
    assert np.mean(got32 != ref64.astype(np.float32)) < 1e-5
