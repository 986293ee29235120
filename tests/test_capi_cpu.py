"""C ABI checks that need no GPU: the library loads, exports every entry point
declared in include/mds.h, validates arguments on the host, sizes the
workspace, and reports MDS_ERR_NO_DEVICE instead of touching a device."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

torch = pytest.importorskip("torch")
mds = pytest.importorskip("paper_1803_02272_amd")
from paper_1803_02272_amd import _capi  # noqa: E402

HEADER = os.path.join(ROOT, "include", "mds.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mds_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = _capi.lib()
    names = declared_functions()
    assert "mds_plan" in names and "mds_run" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(names) <= set(_capi.SIGNATURES), set(names) - set(_capi.SIGNATURES)


def _plan(n, k, p, q, form=1, dt=0, split=0, flags=0):
    L = _capi.lib()
    h = ctypes.c_void_p()
    opts = _capi.MdsOpts(form, dt, split, flags)
    st = L.mds_plan_ex(ctypes.byref(h), n, k, p, q, 0, ctypes.byref(opts))
    return st, h


@pytest.mark.parametrize("n,k,p,q", [(1, 1, 0, 0), (10, 0, 2, 1), (10, 2, -1, 1), (10, 2, 2, -1),
                                     (10, 6, 5, 0), (100000, 200, 57, 2)])
def test_invalid_arguments_rejected(n, k, p, q):
    st, h = _plan(n, k, p, q)
    assert st == _capi.ERR_INVALID_ARG
    assert h.value is None
    assert _capi.lib().mds_last_error().decode()


def test_invalid_options_rejected():
    assert _plan(100, 4, 4, 1, form=7)[0] == _capi.ERR_INVALID_ARG
    assert _plan(100, 4, 4, 1, dt=5)[0] == _capi.ERR_INVALID_ARG
    assert _plan(100, 4, 4, 1, flags=128)[0] == _capi.ERR_INVALID_ARG
    assert _plan(100, 4, 4, 1, split=-1)[0] == _capi.ERR_INVALID_ARG
    for form, flags in ((2, _capi.FLAG_FULL_PROJECTION), (2, _capi.FLAG_FP32_MFMA_PROJECTION),
                        (2, _capi.FLAG_FULL_PROJECTION | _capi.FLAG_FP32_MFMA_PROJECTION),
                        (1, _capi.FLAG_SPLIT_FP32), (1, _capi.FLAG_SPLIT_FP32 | _capi.FLAG_FULL_PROJECTION),
                        (0, _capi.FLAG_FULL_STATS), (2, _capi.FLAG_FULL_STATS | _capi.FLAG_FULL_PROJECTION),
                        (1, _capi.FLAG_CHECK_INPUT), (2, _capi.FLAG_LOWP_ALL_RANGE),
                        (3, _capi.FLAG_LOWP_ALL_RANGE | _capi.FLAG_CHECK_INPUT), (2, _capi.FLAG_FP32_PROJECTION),
                        (3, _capi.FLAG_FP32_PROJECTION | _capi.FLAG_FULL_PROJECTION)):
        st, h = _plan(100, 4, 4, 1, form=form, flags=flags)
        assert st == _capi.OK
        _capi.lib().mds_destroy(h)


def test_workspace_size_scales_with_form():
    L = _capi.lib()
    sizes = {}
    for form in (0, 1, 2):
        st, h = _plan(20000, 50, 10, 2, form=form)
        assert st == _capi.OK
        b = ctypes.c_size_t()
        assert L.mds_workspace_size(h, ctypes.byref(b)) == _capi.OK
        sizes[form] = b.value
        L.mds_destroy(h)
    npad = 20224
    # only the bf16 form stores G (2 bytes per entry); the others recentre D on the fly
    assert sizes[0] < npad * npad and sizes[1] < npad * npad
    assert npad * npad * 2 <= sizes[2] < npad * npad * 3
    # with q = 0 the bf16 form's one range pass is an fp32 pass: no G is stored
    st, h = _plan(20000, 50, 10, 0, form=2)
    b = ctypes.c_size_t()
    assert L.mds_workspace_size(h, ctypes.byref(b)) == _capi.OK and b.value < npad * npad
    L.mds_destroy(h)
    # the input check covers n up to 65535 tiles of 64
    assert _plan(65535 * 64 + 1, 4, 4, 1, flags=_capi.FLAG_CHECK_INPUT)[0] == _capi.ERR_INVALID_ARG


def test_run_without_device_reports_no_device():
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = _capi.lib()
    st, h = _plan(64, 4, 4, 1)
    assert st == _capi.OK
    dummy = ctypes.c_void_p(0x1000)
    assert L.mds_run(h, dummy, dummy, dummy, None) == _capi.ERR_NO_DEVICE
    # argument errors are reported before any device query
    assert L.mds_run(h, None, dummy, dummy, None) == _capi.ERR_INVALID_ARG
    assert L.mds_run_stages(h, dummy, None, None, None, 3, 9) == _capi.ERR_INVALID_ARG
    info = _capi.MdsInfo()
    assert L.mds_get_info(h, ctypes.byref(info), None) == _capi.OK
    assert info.l == 8 and info.l_pad == 16 and info.n == 64 and info.ldg == 256
    buf = _capi.MdsBuffer()
    assert L.mds_get_buffer(h, 0, ctypes.byref(buf)) == _capi.ERR_STATE
    L.mds_destroy(h)


def test_status_strings():
    L = _capi.lib()
    for code in range(-10, 2):
        assert L.mds_status_string(code).decode()
    assert L.mds_version().decode().count(".") == 2


def test_server_without_device_and_bad_arguments():
    L = _capi.lib()
    h = ctypes.c_void_p()
    assert L.mds_server_create(ctypes.byref(h), 1 << 20, 0) == _capi.ERR_INVALID_ARG
    assert L.mds_server_create(ctypes.byref(h), 1 << 20, 1000) == _capi.ERR_INVALID_ARG
    assert L.mds_server_create(ctypes.byref(h), 16, 2) == _capi.ERR_INVALID_ARG
    assert L.mds_server_create(None, 1 << 20, 2) == _capi.ERR_INVALID_ARG
    st = ctypes.c_int()
    assert L.mds_poll(None, 1, ctypes.byref(st), None) == _capi.ERR_INVALID_ARG
    assert L.mds_cancel(None, 1) == _capi.ERR_INVALID_ARG
    t = ctypes.c_uint64()
    assert L.mds_submit(None, None, None, None, None, ctypes.byref(t)) == _capi.ERR_INVALID_ARG
    if not torch.cuda.is_available():
        assert L.mds_server_create(ctypes.byref(h), 1 << 20, 2) == _capi.ERR_NO_DEVICE
        assert h.value is None
