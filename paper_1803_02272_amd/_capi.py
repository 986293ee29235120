"""ctypes binding of the C ABI in include/mds.h (argument marshalling only).

Every computation happens in the HIP library ``libmds.so`` next to this file.
If the library is missing the import fails loudly: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmds.so")

# status codes (mds_status)
OK = 0
PENDING = 1
ERR_INVALID_ARG = -1
ERR_NO_DEVICE = -2
ERR_OOM = -3
ERR_BUDGET = -4
ERR_NONFINITE = -5
ERR_NUMERICAL = -6
ERR_HIP = -7
ERR_CANCELLED = -8
ERR_STATE = -9
ERR_NOT_METRIC = -10

# forms and dtypes
FORM_FP64, FORM_FP32, FORM_BF16, FORM_FP8 = 0, 1, 2, 3
FORMS = {"fp64": FORM_FP64, "fp32": FORM_FP32, "bf16": FORM_BF16, "fp8": FORM_FP8}
DTYPE_F32, DTYPE_F64 = 0, 1

# stages
STAGE_CENTER, STAGE_OMEGA, STAGE_RANGE, STAGE_ALL = 1, 2, 3, 100

# buffers
(BUF_G, BUF_GREF, BUF_ROWMEAN, BUF_COLMEAN, BUF_MEAN, BUF_X, BUF_Q, BUF_Y, BUF_B, BUF_THETA, BUF_V, BUF_W, BUF_T,
 BUF_Q1, BUF_GSCALE) = range(15)

MAX_L = 256
BATCH_STATIC_BYTES = 128 << 20  # MDS_BATCH_STATIC_BYTES

# option flags (mds_opts.flags)
FLAG_FULL_PROJECTION = 1
FLAG_FP32_MFMA_PROJECTION = 2
FLAG_SPLIT_FP32 = 4
FLAG_FULL_STATS = 8
FLAG_CHECK_INPUT = 16
FLAG_LOWP_ALL_RANGE = 32
FLAG_FP32_PROJECTION = 64
CC_FULL_MATRIX = 1


class MdsOpts(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("d_dtype", ctypes.c_int32),
                ("gpass_split", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("proj_split", ctypes.c_int32), ("write_split", ctypes.c_int32),
                ("f32_split", ctypes.c_int32)]


class MdsBuffer(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("rows", ctypes.c_int64), ("cols", ctypes.c_int64), ("ld", ctypes.c_int64)]


class MdsInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("nonfinite", ctypes.c_int32),
                ("orth_fallbacks", ctypes.c_int32), ("jacobi_sweeps", ctypes.c_int32),
                ("jacobi_unconverged", ctypes.c_int32), ("rank_deficient", ctypes.c_int32),
                ("k", ctypes.c_int32), ("l", ctypes.c_int32), ("l_pad", ctypes.c_int32),
                ("q", ctypes.c_int32), ("form", ctypes.c_int32), ("gpass_split", ctypes.c_int32),
                ("n", ctypes.c_int64), ("ldg", ctypes.c_int64),
                ("sum_sq", ctypes.c_double), ("frob2", ctypes.c_double), ("trace", ctypes.c_double),
                ("asym_pairs", ctypes.c_int64), ("diag_nonzero", ctypes.c_int64),
                ("tuned_from_cache", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


PHASES = ["stats", "write", "omega", "gpass", "reduce", "orth", "gpass_ref", "small", "coords", "gpass_f32",
          "check"]


class MdsPhaseTime(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("total_ms", ctypes.c_float), ("min_ms", ctypes.c_float),
                ("max_ms", ctypes.c_float)]


class MdsBatchJob(ctypes.Structure):
    _fields_ = [("D", ctypes.c_void_p), ("coords", ctypes.c_void_p), ("eigvals", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("k", ctypes.c_int32), ("oversample", ctypes.c_int32),
                ("q", ctypes.c_int32), ("d_dtype", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class MdsTuneResult(ctypes.Structure):
    _fields_ = [("range_split", ctypes.c_int32), ("proj_split", ctypes.c_int32), ("write_split", ctypes.c_int32),
                ("f32_split", ctypes.c_int32), ("range_ms", ctypes.c_float), ("proj_ms", ctypes.c_float),
                ("write_ms", ctypes.c_float), ("f32_ms", ctypes.c_float), ("candidates", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "pad_"}


class MdsBatchTune(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("pad_", ctypes.c_int32), ("batch_ms_per_job", ctypes.c_float * 3),
                ("batch_ms_best", ctypes.c_float), ("plan_ms", ctypes.c_float)]


class MdsJobTimes(ctypes.Structure):
    _fields_ = [("queue_ms", ctypes.c_double), ("run_ms", ctypes.c_double), ("latency_ms", ctypes.c_double)]


class MdsServerInfo(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int32), ("running", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("completed", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("budget_bytes", ctypes.c_size_t),
                ("used_bytes", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "pad_"}


# exported symbol -> (restype, argtypes)
SIGNATURES = {
    "mds_plan": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int64, ctypes.c_int32,
                                ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64]),
    "mds_plan_ex": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int64, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.POINTER(MdsOpts)]),
    "mds_workspace_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "mds_set_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "mds_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p]),
    "mds_run_stages": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "mds_get_buffer": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(MdsBuffer)]),
    "mds_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(MdsInfo), ctypes.c_void_p]),
    "mds_set_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "mds_get_timings": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(MdsPhaseTime), ctypes.c_void_p]),
    "mds_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.POINTER(MdsTuneResult)]),
    "mds_destroy": (None, [ctypes.c_void_p]),
    "mds_philox4x64_10": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "mds_hamming_distances": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_void_p, ctypes.c_void_p]),
    "mds_euclidean_distances": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                               ctypes.c_void_p, ctypes.c_void_p]),
    "mds_threshold_components": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                                ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mds_batch_workspace_size": (ctypes.c_int, [ctypes.POINTER(MdsBatchJob), ctypes.c_int32, ctypes.c_int32,
                                                ctypes.POINTER(ctypes.c_size_t)]),
    "mds_run_batch": (ctypes.c_int, [ctypes.POINTER(MdsBatchJob), ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.c_size_t, ctypes.c_int32, ctypes.c_void_p]),
    "mds_autotune_batch": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.POINTER(MdsBatchTune)]),
    "mds_server_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "mds_batch_status": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.c_void_p]),
    "mds_run_batch_static": (ctypes.c_int, [ctypes.POINTER(MdsBatchJob), ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "mds_server_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t, ctypes.c_int32]),
    "mds_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "mds_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(MdsJobTimes)]),
    "mds_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(MdsJobTimes)]),
    "mds_cancel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "mds_server_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(MdsServerInfo)]),
    "mds_server_set_batching": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32]),
    "mds_server_destroy": (None, [ctypes.c_void_p]),
    "mds_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "mds_last_error": (ctypes.c_char_p, []),
    "mds_version": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libmds.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        # torch first: its bundled HIP runtime (SONAME libamdhip64.so.7) then
        # satisfies libmds.so's dependency, so the process holds one runtime
        # and torch's streams and allocations are valid in the library.
        import torch  # noqa: F401

        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class MdsError(RuntimeError):
    def __init__(self, status, where):
        L = lib()
        msg = L.mds_last_error().decode()
        super().__init__(f"{where}: {L.mds_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def check(status, where):
    if status != OK:
        raise MdsError(status, where)
    return status
