"""MI355X-native random-projection classical MDS.

Python face of the HIP library ``libmds.so`` (C ABI in include/mds.h).  This
module marshals arguments only: PyTorch supplies device memory and the
stream; every step of the method runs in the library's kernels.

    import torch, paper_1803_02272_amd as mds
    plan = mds.Plan(n, k=100, oversample=20, q=2, seed=0, form="bf16")
    coords, eigvals = plan.run(D)      # D: torch.cuda float32 n x n
"""
from __future__ import annotations

import ctypes

from . import _capi
from ._capi import MdsError, check

__all__ = ["Plan", "MdsError", "library_version", "FORMS", "hamming_distances", "euclidean_distances",
           "threshold_components"]

FORMS = _capi.FORMS


def library_version() -> str:
    return _capi.lib().mds_version().decode()


def _stream_handle(stream):
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _distance_out(n, dtype, out):
    import torch

    tdt = {"f32": torch.float32, "f64": torch.float64}[dtype]
    if out is None:
        out = torch.empty((n, n), dtype=tdt, device="cuda")
    if out.dtype != tdt or tuple(out.shape) != (n, n) or not out.is_contiguous() or not out.is_cuda:
        raise ValueError("out must be a contiguous CUDA tensor of shape (n, n) and the requested dtype")
    return out, (_capi.DTYPE_F64 if dtype == "f64" else _capi.DTYPE_F32)


def hamming_distances(codes, dtype="f32", out=None, stream=None):
    """D[i, j] = (positions where reads i and j differ) / length
    (mds_hamming_distances).  codes: CUDA uint8 tensor n x length of base
    codes 0..3; returns (or fills) the n x n D in fp32 or fp64."""
    import torch

    if codes.dtype != torch.uint8 or codes.dim() != 2 or not codes.is_cuda:
        raise ValueError("codes must be a CUDA uint8 tensor of shape (n, length)")
    codes = codes.contiguous()
    n, length = codes.shape
    out, dt = _distance_out(n, dtype, out)
    check(_capi.lib().mds_hamming_distances(ctypes.c_void_p(codes.data_ptr()), n, length, dt,
                                            ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
          "mds_hamming_distances")
    return out


def threshold_components(D, threshold, full_matrix=False, stream=None):
    """Connected components of the graph with an edge (i, j) wherever
    D[i, j] <= threshold (mds_threshold_components).  D: CUDA float32 or
    float64 n x n (upper triangle read unless full_matrix).  Returns
    (labels, count): CUDA int32 labels (the smallest index of each item's
    component) and a CUDA int64 scalar tensor, both filled on the stream."""
    import torch

    if D.dim() != 2 or D.shape[0] != D.shape[1] or not D.is_cuda or D.dtype not in (torch.float32, torch.float64):
        raise ValueError("D must be a square CUDA float32/float64 tensor")
    D = D.contiguous()
    n = D.shape[0]
    labels = torch.empty(n, dtype=torch.int32, device=D.device)
    count = torch.empty((), dtype=torch.int64, device=D.device)
    dt = _capi.DTYPE_F64 if D.dtype == torch.float64 else _capi.DTYPE_F32
    check(_capi.lib().mds_threshold_components(ctypes.c_void_p(D.data_ptr()), dt, n, float(threshold),
                                               _capi.CC_FULL_MATRIX if full_matrix else 0,
                                               ctypes.c_void_p(labels.data_ptr()), ctypes.c_void_p(count.data_ptr()),
                                               _stream_handle(stream)),
          "mds_threshold_components")
    return labels, count


def euclidean_distances(X, dtype="f32", out=None, stream=None):
    """D[i, j] = sqrt(sum_k (x_ik - x_jk)^2) in fp64, rounded to the output
    type (mds_euclidean_distances).  X: CUDA float64 tensor n x dim."""
    import torch

    if X.dtype != torch.float64 or X.dim() != 2 or not X.is_cuda:
        raise ValueError("X must be a CUDA float64 tensor of shape (n, dim)")
    X = X.contiguous()
    n, dim = X.shape
    out, dt = _distance_out(n, dtype, out)
    check(_capi.lib().mds_euclidean_distances(ctypes.c_void_p(X.data_ptr()), n, dim, dt,
                                              ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
          "mds_euclidean_distances")
    return out


class Plan:
    """A plan for one problem shape: n points, k axes, oversample p, q power
    iterations, test-matrix seed, G-pass form ("fp64" | "fp32" | "bf16") and
    the dtype of D ("f32" | "f64").  full_projection=True streams all of G in
    the projection pass instead of its upper triangle (MDS_FLAG_FULL_PROJECTION);
    fp32_mfma_projection=True runs the bf16/fp8 forms' projection as an fp32
    pass on fp32 MFMA (MDS_FLAG_FP32_MFMA_PROJECTION);
    split_fp32=True runs every pass of the fp32 form as that split
    (MDS_FLAG_SPLIT_FP32); full_stats=True reads all of D in the centring
    statistics instead of its upper-triangle tiles (MDS_FLAG_FULL_STATS);
    check_input=True tests that D is symmetric with a zero diagonal
    (MDS_FLAG_CHECK_INPUT; info() then reports asym_pairs and diag_nonzero
    and status ERR_NOT_METRIC on a violation); lowp_all_range=True runs every
    range pass of the bf16/fp8 forms on the stored low-precision G, without
    the 16-bit first and last range passes (MDS_FLAG_LOWP_ALL_RANGE);
    fp32_projection=True makes the bf16/fp8 forms' projection an fp32 pass
    (three-term split) instead of a 16-bit one (MDS_FLAG_FP32_PROJECTION)."""

    def __init__(self, n, k, oversample=10, q=2, seed=0, form="fp32", d_dtype="f32", gpass_split=0,
                 workspace="torch", full_projection=False, proj_split=0, write_split=0,
                 fp32_mfma_projection=False, split_fp32=False, full_stats=False, check_input=False,
                 lowp_all_range=False, f32_split=0, fp32_projection=False):
        L = _capi.lib()
        self.n, self.k, self.oversample, self.q, self.seed = int(n), int(k), int(oversample), int(q), int(seed)
        self.form = form
        self.d_dtype = d_dtype
        opts = _capi.MdsOpts(FORMS[form] if isinstance(form, str) else int(form),
                             _capi.DTYPE_F64 if d_dtype in ("f64", "float64") else _capi.DTYPE_F32,
                             int(gpass_split),
                             (_capi.FLAG_FULL_PROJECTION if full_projection else 0)
                             | (_capi.FLAG_FP32_MFMA_PROJECTION if fp32_mfma_projection else 0)
                             | (_capi.FLAG_SPLIT_FP32 if split_fp32 else 0)
                             | (_capi.FLAG_FULL_STATS if full_stats else 0)
                             | (_capi.FLAG_CHECK_INPUT if check_input else 0)
                             | (_capi.FLAG_LOWP_ALL_RANGE if lowp_all_range else 0)
                             | (_capi.FLAG_FP32_PROJECTION if fp32_projection else 0),
                             int(proj_split), int(write_split), int(f32_split))
        h = ctypes.c_void_p()
        check(L.mds_plan_ex(ctypes.byref(h), self.n, self.k, self.oversample, self.q, self.seed,
                            ctypes.byref(opts)), "mds_plan_ex")
        self._h = h
        self._ws = None
        self._workspace_mode = workspace

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _capi.lib().mds_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self):
        return self._h

    def autotune(self, D, stream=None):
        """Time the split-K candidates of each pass kind on D and keep the
        fastest (call before the first run); returns the chosen splits."""
        self._check_D(D)
        r = _capi.MdsTuneResult()
        check(_capi.lib().mds_autotune(self._h, ctypes.c_void_p(D.data_ptr()), _stream_handle(stream),
                                       ctypes.byref(r)), "mds_autotune")
        return r.as_dict()

    # -- workspace -----------------------------------------------------------
    def workspace_size(self) -> int:
        b = ctypes.c_size_t()
        check(_capi.lib().mds_workspace_size(self._h, ctypes.byref(b)), "mds_workspace_size")
        return int(b.value)

    def attach_workspace(self, device=None):
        """Allocate the workspace with PyTorch and hand it to the library."""
        import torch

        if self._ws is None:
            nbytes = self.workspace_size()
            ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device or "cuda")
            off = (-ws.data_ptr()) % 256
            check(_capi.lib().mds_set_workspace(self._h, ctypes.c_void_p(ws.data_ptr() + off), nbytes),
                  "mds_set_workspace")
            self._ws = ws
        return self._ws

    # -- runs ----------------------------------------------------------------
    def _check_D(self, D):
        import torch

        want = torch.float64 if self.d_dtype in ("f64", "float64") else torch.float32
        if not (D.is_cuda and D.dtype == want and D.dim() == 2 and D.shape[0] == self.n
                and D.shape[1] == self.n and D.is_contiguous()):
            raise ValueError(f"D must be a contiguous cuda {want} tensor of shape ({self.n}, {self.n})")

    def run(self, D, coords=None, eigvals=None, stream=None):
        """Enqueue the full method; returns (coords n x k fp64, eigvals k fp64)."""
        import torch

        self._check_D(D)
        if self._workspace_mode == "torch":
            self.attach_workspace(D.device)
        if coords is None:
            coords = torch.empty((self.n, self.k), dtype=torch.float64, device=D.device)
        if eigvals is None:
            eigvals = torch.empty((self.k,), dtype=torch.float64, device=D.device)
        check(_capi.lib().mds_run(self._h, ctypes.c_void_p(D.data_ptr()), ctypes.c_void_p(coords.data_ptr()),
                                  ctypes.c_void_p(eigvals.data_ptr()), _stream_handle(stream)), "mds_run")
        return coords, eigvals

    def run_stages(self, D, stop_after, range_passes=0, coords=None, eigvals=None, stream=None):
        self._check_D(D)
        if self._workspace_mode == "torch":
            self.attach_workspace(D.device)
        cp = ctypes.c_void_p(coords.data_ptr()) if coords is not None else None
        ep = ctypes.c_void_p(eigvals.data_ptr()) if eigvals is not None else None
        check(_capi.lib().mds_run_stages(self._h, ctypes.c_void_p(D.data_ptr()), cp, ep, _stream_handle(stream),
                                         int(stop_after), int(range_passes)), "mds_run_stages")

    def buffer(self, which):
        """View of an internal buffer (valid once the stream work that wrote
        it has completed) as a torch tensor of its logical shape.  Needs the
        torch-allocated workspace."""
        import torch

        if self._ws is None:
            raise RuntimeError("buffer() needs a workspace attached with attach_workspace()")
        b = _capi.MdsBuffer()
        check(_capi.lib().mds_get_buffer(self._h, int(which), ctypes.byref(b)), "mds_get_buffer")
        dt = {0: torch.float64, 1: torch.float32, 2: torch.bfloat16, 3: torch.float8_e4m3fn}[b.dtype]
        esz = {0: 8, 1: 4, 2: 2, 3: 1}[b.dtype]
        rows, cols, ld = b.rows, b.cols, b.ld
        total = (rows - 1) * ld + cols if rows > 0 else 0
        off = b.ptr - self._ws.data_ptr()
        if off < 0 or off + total * esz > self._ws.numel():
            raise RuntimeError("buffer outside the workspace")
        flat = self._ws[off: off + total * esz].view(dt)
        return flat.as_strided((rows, cols), (ld, 1))

    def set_timing(self, enable=True):
        check(_capi.lib().mds_set_timing(self._h, 1 if enable else 0), "mds_set_timing")

    def timings(self, stream=None):
        """{phase: (count, total_ms, min_ms, max_ms)} since the last call (syncs the stream)."""
        arr = (_capi.MdsPhaseTime * len(_capi.PHASES))()
        check(_capi.lib().mds_get_timings(self._h, arr, _stream_handle(stream)), "mds_get_timings")
        return {name: (t.count, t.total_ms, t.min_ms, t.max_ms) for name, t in zip(_capi.PHASES, arr)}

    def info(self, stream=None):
        inf = _capi.MdsInfo()
        check(_capi.lib().mds_get_info(self._h, ctypes.byref(inf), _stream_handle(stream)), "mds_get_info")
        return inf.as_dict()


def run_batch(problems, form="bf16", stream=None, tile=0):
    """Batched small instances in one persistent launch (mds_run_batch).

    problems: list of dicts with keys D (contiguous cuda float32/float64 n x n),
    k, oversample, q, seed.  Returns (results, statuses) with results a list
    of (coords n x k, eigvals k) fp64 tensors; synchronises the stream."""
    import torch

    fk = FORMS[form] if isinstance(form, str) else int(form)
    arr = (_capi.MdsBatchJob * max(len(problems), 1))()
    outs = []
    for i, pr in enumerate(problems):
        D = pr["D"]
        n = D.shape[0]
        if not (D.is_cuda and D.dim() == 2 and D.shape[1] == n and D.is_contiguous()
                and D.dtype in (torch.float32, torch.float64)):
            raise ValueError("D must be a contiguous square cuda float32/float64 tensor")
        c = torch.empty((n, int(pr["k"])), dtype=torch.float64, device=D.device)
        e = torch.empty((int(pr["k"]),), dtype=torch.float64, device=D.device)
        outs.append((c, e))
        arr[i] = _capi.MdsBatchJob(D.data_ptr(), c.data_ptr(), e.data_ptr(), n, int(pr["k"]),
                                   int(pr.get("oversample", 10)), int(pr.get("q", 2)),
                                   _capi.DTYPE_F64 if D.dtype == torch.float64 else _capi.DTYPE_F32,
                                   int(pr.get("seed", 0)))
    L = _capi.lib()
    nb = ctypes.c_size_t()
    check(L.mds_batch_workspace_size(arr, len(problems), fk, ctypes.byref(nb)), "mds_batch_workspace_size")
    ws = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    wp = ctypes.c_void_p(ws.data_ptr() + off)
    sh = _stream_handle(stream)
    check(L.mds_run_batch(arr, len(problems), fk, wp, nb.value, int(tile), sh), "mds_run_batch")
    st = (ctypes.c_int32 * max(len(problems), 1))()
    check(L.mds_batch_status(wp, len(problems), st, sh), "mds_batch_status")
    return outs, [int(st[i]) for i in range(len(problems))]


def autotune_batch(n, k=20, oversample=10, q=2, form="bf16", batch=32, stream=None):
    """Time the batched kernel's tile shapes (and the plan path) at size n;
    the fastest tile is recorded for mds_run_batch.  Returns a dict."""
    fk = FORMS[form] if isinstance(form, str) else int(form)
    t = _capi.MdsBatchTune()
    check(_capi.lib().mds_autotune_batch(fk, int(n), int(k), int(oversample), int(q), int(batch),
                                         _stream_handle(stream), ctypes.byref(t)), "mds_autotune_batch")
    return {"tile": t.tile, "batch_ms_per_job": list(t.batch_ms_per_job), "batch_ms_best": t.batch_ms_best,
            "plan_ms": t.plan_ms}


class Server:
    """Continuous-batching server (mds_server_*): a device arena of
    ``budget_bytes`` and ``slots`` concurrent streams.  ``submit`` queues a job
    of a Plan on a device D and returns a ticket; ``poll`` never blocks and
    returns None while the job is pending, else (status, times)."""

    def __init__(self, budget_bytes, slots=8, small_n_max=None, max_batch=None):
        h = ctypes.c_void_p()
        check(_capi.lib().mds_server_create(ctypes.byref(h), int(budget_bytes), int(slots)), "mds_server_create")
        self._h = h
        self._keep = {}  # ticket -> tensors that must outlive the job
        if small_n_max is not None or max_batch is not None:
            self.set_batching(2048 if small_n_max is None else small_n_max, 32 if max_batch is None else max_batch)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _capi.lib().mds_server_destroy(self._h)
            self._h = None
        self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def submit(self, plan, D, coords=None, eigvals=None):
        """Queue plan on D; returns (ticket, coords, eigvals) with the outputs
        filled in once the job completes."""
        import torch

        plan._check_D(D)
        if coords is None:
            coords = torch.empty((plan.n, plan.k), dtype=torch.float64, device=D.device)
        if eigvals is None:
            eigvals = torch.empty((plan.k,), dtype=torch.float64, device=D.device)
        t = ctypes.c_uint64()
        check(_capi.lib().mds_submit(self._h, plan.handle, ctypes.c_void_p(D.data_ptr()),
                                     ctypes.c_void_p(coords.data_ptr()), ctypes.c_void_p(eigvals.data_ptr()),
                                     ctypes.byref(t)), "mds_submit")
        self._keep[t.value] = (D, coords, eigvals)
        return t.value, coords, eigvals

    def _done(self, ticket, st, tm):
        self._keep.pop(ticket, None)
        return st.value, {"queue_ms": tm.queue_ms, "run_ms": tm.run_ms, "latency_ms": tm.latency_ms}

    def poll(self, ticket):
        st = ctypes.c_int()
        tm = _capi.MdsJobTimes()
        check(_capi.lib().mds_poll(self._h, int(ticket), ctypes.byref(st), ctypes.byref(tm)), "mds_poll")
        if st.value == _capi.PENDING:
            return None
        return self._done(ticket, st, tm)

    def wait(self, ticket):
        st = ctypes.c_int()
        tm = _capi.MdsJobTimes()
        check(_capi.lib().mds_wait(self._h, int(ticket), ctypes.byref(st), ctypes.byref(tm)), "mds_wait")
        return self._done(ticket, st, tm)

    def cancel(self, ticket):
        check(_capi.lib().mds_cancel(self._h, int(ticket)), "mds_cancel")

    def set_batching(self, small_n_max=2048, max_batch=32):
        """Small jobs (n <= small_n_max, l_pad <= 64) at the queue head run
        together as one batched launch; small_n_max=0 turns batching off."""
        check(_capi.lib().mds_server_set_batching(self._h, int(small_n_max), int(max_batch)),
              "mds_server_set_batching")

    def autotune(self, form="bf16", k=20, oversample=10, q=2):
        """Choose the batching threshold (and batched tile shapes) by timing; returns small_n_max."""
        fk = FORMS[form] if isinstance(form, str) else int(form)
        v = ctypes.c_int64()
        check(_capi.lib().mds_server_autotune(self._h, fk, int(k), int(oversample), int(q), ctypes.byref(v)),
              "mds_server_autotune")
        return int(v.value)

    def stats(self):
        inf = _capi.MdsServerInfo()
        check(_capi.lib().mds_server_stats(self._h, ctypes.byref(inf)), "mds_server_stats")
        return inf.as_dict()
