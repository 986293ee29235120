"""mds_run_batch_static: the allocation-free batch entry point (static device
scratch) against mds_run_batch on the same jobs, through the C ABI.  Two
calls in a row, the second with a smaller batch, each compared bit for bit
with the workspace path (same kernels, same per-instance arithmetic); the
statuses the kernel writes match mds_batch_status; an oversized batch is
refused on the host."""
import ctypes

import numpy as np
import pytest

import workloads as W
from gpu_util import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1803_02272_amd as mds  # noqa: E402
from paper_1803_02272_amd import _capi  # noqa: E402


def _dist(kind, n, seed):
    if kind == "gm":
        X, _ = W.gaussian_mixture(n, 50, 10, 25.0, seed)
        return W.euclidean_distances(X, dtype=np.float32)
    reads, _ = W.amplicon_reads(n, 50, seed=seed)
    return W.hamming_distances(reads)


def _jobs(specs, with_nan=None):
    Ds, arr, outs_a, outs_b = [], (_capi.MdsBatchJob * len(specs))(), [], []
    for i, (kind, n, k, p, q, seed) in enumerate(specs):
        D = torch.from_numpy(_dist(kind, n, seed)).cuda()
        if with_nan == i:
            D[2, 5] = float("nan")
        Ds.append(D)
        ca = torch.full((n, k), -7.0, dtype=torch.float64, device="cuda")
        ea = torch.full((k,), -7.0, dtype=torch.float64, device="cuda")
        outs_a.append((ca, ea))
        outs_b.append((torch.full_like(ca, -9.0), torch.full_like(ea, -9.0)))
        arr[i] = _capi.MdsBatchJob(D.data_ptr(), ca.data_ptr(), ea.data_ptr(), n, k, p, q, _capi.DTYPE_F32, seed)
    return Ds, arr, outs_a, outs_b


def _run_both(specs, form, with_nan=None):
    L = _capi.lib()
    fk = _capi.FORMS[form]
    Ds, arr, outs_a, outs_b = _jobs(specs, with_nan)
    count = len(specs)
    # workspace path
    nb = ctypes.c_size_t()
    assert L.mds_batch_workspace_size(arr, count, fk, ctypes.byref(nb)) == _capi.OK
    assert nb.value <= _capi.BATCH_STATIC_BYTES
    ws = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
    wp = ctypes.c_void_p(ws.data_ptr() + (-ws.data_ptr()) % 256)
    assert L.mds_run_batch(arr, count, fk, wp, nb.value, 4, None) == _capi.OK
    st_a = (ctypes.c_int32 * count)()
    assert L.mds_batch_status(wp, count, st_a, None) == _capi.OK
    # allocation-free path, same jobs with the second set of outputs
    for i, (cb, eb) in enumerate(outs_b):
        arr[i].coords, arr[i].eigvals = cb.data_ptr(), eb.data_ptr()
    st_dev = torch.full((count,), 12345, dtype=torch.int32, device="cuda")
    assert L.mds_run_batch_static(arr, count, fk, 4, ctypes.c_void_p(st_dev.data_ptr()), None) == _capi.OK
    torch.cuda.synchronize()
    assert st_dev.cpu().tolist() == list(st_a)
    for (ca, ea), (cb, eb) in zip(outs_a, outs_b):  # bit for bit (a NaN instance included)
        assert torch.equal(ca.view(torch.int64), cb.view(torch.int64))
        assert torch.equal(ea.view(torch.int64), eb.view(torch.int64))
    return list(st_a)


@pytest.mark.parametrize("form", ["bf16", "fp64"])
def test_static_batch_matches_workspace_batch_twice(form):
    count = 24 if form == "bf16" else 12  # fp64 G takes four times the bytes of bf16 G
    first = [("gm" if i % 2 else "amp", 300 + 37 * i, 20 if i % 3 else 8, 10, 2 if i % 4 else 1, 50 + i)
             for i in range(count)]
    second = [("amp", 130 + 11 * i, 6, 4, 1, 900 + i) for i in range(5)]  # smaller batch, smaller instances
    say(f"[no-alloc] form={form}: {len(first)} instances, then {len(second)}")
    assert _run_both(first, form) == [0] * len(first)
    st = _run_both(second, form, with_nan=2)
    assert st[2] == _capi.ERR_NONFINITE and st[:2] + st[3:] == [0] * 4


def test_static_batch_rejects_oversized_batch():
    L = _capi.lib()
    arr = (_capi.MdsBatchJob * 40)()
    for i in range(40):  # about 9.5 MB of workspace each in the bf16 form
        arr[i] = _capi.MdsBatchJob(256, 256, 256, 2048, 20, 10, 2, _capi.DTYPE_F32, i)
    nb = ctypes.c_size_t()
    assert L.mds_batch_workspace_size(arr, 40, _capi.FORM_BF16, ctypes.byref(nb)) == _capi.OK
    assert nb.value > _capi.BATCH_STATIC_BYTES
    assert L.mds_run_batch_static(arr, 40, _capi.FORM_BF16, 0, None, None) == _capi.ERR_INVALID_ARG
    assert b"static scratch" in L.mds_last_error()
