"""The library's threshold-graph components (mds_threshold_components;
Sec. 7, Conclusions and perspectives) against the CPU oracle: labels (the
smallest index of each component) and counts must be identical.  Small and
ragged sizes (partial tiles), fp32 and fp64 D, aligned and unaligned D, the
empty and the complete graph, NaN entries, an asymmetric D in both reading
modes, planted clusters, and at full size (n = 100,000 reads) the labels
against scipy's connected_components on the edges of D fetched row block by
row block."""
import time

import numpy as np
import pytest

import workloads as W
from gpu_util import say
from oracle import components as OC

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1803_02272_amd as mds  # noqa: E402
from paper_1803_02272_amd import _capi  # noqa: E402


def random_symmetric(n, seed, dtype):
    rng = np.random.default_rng(seed)
    A = np.triu(rng.random((n, n)), 1)
    return (A + A.T).astype(dtype)


def run(D, theta, full=False):
    lab, cnt = mds.threshold_components(torch.from_numpy(np.ascontiguousarray(D)).cuda(), theta, full_matrix=full)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), int(cnt.item())


@pytest.mark.parametrize("n,theta", [(1, 0.5), (2, 0.3), (5, 0.2), (129, 0.02), (1000, 0.0012), (1000, 0.002),
                                     (2000, 0.0009)])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_components_match_oracle(n, theta, dtype):
    say(f"[cc] n={n} theta={theta} dtype={np.dtype(dtype).name}")
    D = random_symmetric(n, n, dtype)
    want, wc = OC.threshold_components(D, theta)
    lab, cnt = run(D, theta)
    say(f"    components {cnt} (oracle {wc})")
    assert cnt == wc and np.array_equal(lab, want)


def test_empty_complete_nan_and_asymmetric():
    D = random_symmetric(300, 4, np.float32)
    lab, cnt = run(D, -1.0)
    assert cnt == 300 and np.array_equal(lab, np.arange(300))
    lab, cnt = run(D, 2.0)
    assert cnt == 1 and np.all(lab == 0)
    Dn = D.copy()
    Dn[:, 131] = np.nan
    Dn[131, :] = np.nan
    want, wc = OC.threshold_components(Dn, 2.0)
    lab, cnt = run(Dn, 2.0)
    assert cnt == wc == 2 and np.array_equal(lab, want)
    # an asymmetric D: default reads j > i only, the full mode both triangles
    rng = np.random.default_rng(5)
    A = rng.random((257, 257)).astype(np.float32)
    for full in (False, True):
        want, wc = OC.threshold_components(A, 0.004, full=full)
        lab, cnt = run(A, 0.004, full=full)
        assert cnt == wc and np.array_equal(lab, want), full


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_unaligned_d(dtype):
    n = 301
    D = random_symmetric(n, 7, np.float32 if dtype == torch.float32 else np.float64)
    want, wc = OC.threshold_components(D, 0.004)
    flat = torch.zeros(n * n + 1, dtype=dtype, device="cuda")
    view = flat[1:].view(n, n)
    view.copy_(torch.from_numpy(D))
    labels = torch.empty(n, dtype=torch.int32, device="cuda")
    count = torch.empty((), dtype=torch.int64, device="cuda")
    st = _capi.lib().mds_threshold_components(view.data_ptr(), 0 if dtype == torch.float32 else 1, n, 0.004, 0,
                                              labels.data_ptr(), count.data_ptr(), None)
    assert st == _capi.OK
    torch.cuda.synchronize()
    assert int(count.item()) == wc and np.array_equal(labels.cpu().numpy(), want)


def test_planted_clusters_from_library_distances():
    reads, parent = W.amplicon_reads(3000, 40, rate_lo=0.01, rate_hi=0.03, length=400, seed=2)
    D = mds.hamming_distances(torch.from_numpy(reads).cuda())
    lab, cnt = mds.threshold_components(D, 0.25)
    want, wc = OC.threshold_components(D.cpu().numpy(), 0.25)
    assert int(cnt.item()) == wc == len(np.unique(parent))
    assert np.array_equal(lab.cpu().numpy(), want)


def test_argument_errors():
    L = _capi.lib()
    d = torch.zeros(4, dtype=torch.float32, device="cuda")
    lab = torch.zeros(2, dtype=torch.int32, device="cuda")
    assert L.mds_threshold_components(None, 0, 2, 0.5, 0, lab.data_ptr(), None, None) == _capi.ERR_INVALID_ARG
    assert L.mds_threshold_components(d.data_ptr(), 0, 2, 0.5, 0, None, None, None) == _capi.ERR_INVALID_ARG
    assert L.mds_threshold_components(d.data_ptr(), 2, 2, 0.5, 0, lab.data_ptr(), None, None) == _capi.ERR_INVALID_ARG
    assert L.mds_threshold_components(d.data_ptr(), 0, 2, 0.5, 2, lab.data_ptr(), None, None) == _capi.ERR_INVALID_ARG
    assert L.mds_threshold_components(d.data_ptr(), 0, 2, float("nan"), 0, lab.data_ptr(), None,
                                      None) == _capi.ERR_INVALID_ARG
    # without a count pointer
    assert L.mds_threshold_components(d.data_ptr(), 0, 2, 0.5, 0, lab.data_ptr(), None, None) == _capi.OK
    torch.cuda.synchronize()
    assert lab.cpu().tolist() == [0, 0]


@pytest.mark.slow
def test_full_size_against_scipy_on_fetched_edges():
    csgraph = pytest.importorskip("scipy.sparse.csgraph")
    sparse = pytest.importorskip("scipy.sparse")
    n, theta = 100000, 0.03
    reads, _ = W.amplicon_reads(n, 200, seed=0)
    D = mds.hamming_distances(torch.from_numpy(reads).cuda())
    mds.threshold_components(D, theta)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    lab, cnt = mds.threshold_components(D, theta)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    say(f"[cc full] n={n}: {ms:.2f} ms ({n * (n - 1) / 2 * 4 / ms / 1e6:.0f} GB/s of the upper triangle), "
        f"{int(cnt.item())} components")
    t0 = time.time()
    rows, cols = [], []
    blk = 2000
    for a in range(0, n, blk):
        Db = D[a:a + blk].cpu().numpy()
        ii, jj = np.nonzero(Db <= theta)
        ii = ii + a
        keep = jj > ii
        rows.append(ii[keep])
        cols.append(jj[keep])
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    A = sparse.coo_matrix((np.ones(len(rows), dtype=np.int8), (rows, cols)), shape=(n, n)).tocsr()
    k, sl = csgraph.connected_components(A, directed=False)
    first = np.full(k, n, dtype=np.int64)
    np.minimum.at(first, sl, np.arange(n))
    want = first[sl].astype(np.int32)
    say(f"    {len(rows)} edges fetched, scipy: {k} components ({time.time() - t0:.0f} s)")
    assert int(cnt.item()) == k
    assert np.array_equal(lab.cpu().numpy(), want)
