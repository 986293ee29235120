"""Device-side generation of the synthetic distance matrices (same recipes as
the numpy generators in this package, bit-identical for Hamming distances).
Used for the large inputs of the benchmark and of full-size checks."""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import READ_LENGTH, amplicon_reads, gaussian_mixture, pack_bitplanes

HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


def _load():
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (one HIP runtime: torch's)

        path = os.path.join(HERE, "libmds_gen.so")
        if not os.path.exists(path):
            raise ImportError(f"{path} missing: run workloads/gpu_build.py")
        L = ctypes.CDLL(path)
        L.gen_hamming_f32.restype = ctypes.c_int
        L.gen_hamming_f32.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]
        L.gen_euclid.restype = ctypes.c_int
        L.gen_euclid.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                 ctypes.c_void_p]
        _lib = L
    return _lib


def hamming_from_reads(reads: np.ndarray, out=None):
    """float32 n x n Hamming distance matrix of `reads` on the current device."""
    import torch

    reads = np.asarray(reads, dtype=np.uint8)
    n, L = reads.shape
    planes = torch.from_numpy(pack_bitplanes(reads)).cuda()
    words = planes.shape[2]
    table = torch.from_numpy((np.arange(L + 1, dtype=np.float64) / float(L)).astype(np.float32)[::-1].copy())
    # table[matches] = (L - matches) / L
    table = table.cuda()
    if out is None:
        out = torch.empty((n, n), dtype=torch.float32, device="cuda")
    rc = _load().gen_hamming_f32(ctypes.c_void_p(planes.data_ptr()), n, words, L,
                                 ctypes.c_void_p(table.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != 0:
        raise RuntimeError(f"gen_hamming_f32 failed ({rc})")
    torch.cuda.synchronize()
    return out


def amplicon_distances(n_reads, n_refs, seed=0, length=READ_LENGTH):
    reads, _ = amplicon_reads(n_reads, n_refs, seed=seed, length=length)
    return hamming_from_reads(reads)


def euclidean_from_points(X: np.ndarray, dtype="f32", out=None):
    import torch

    X = np.ascontiguousarray(X, dtype=np.float64)
    n, dim = X.shape
    xt = torch.from_numpy(X).cuda()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if out is None:
        out = torch.empty((n, n), dtype=tdt, device="cuda")
    rc = _load().gen_euclid(ctypes.c_void_p(xt.data_ptr()), n, dim, 1 if dtype == "f64" else 0,
                            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != 0:
        raise RuntimeError(f"gen_euclid failed ({rc})")
    torch.cuda.synchronize()
    return out


def mixture_distances(n, dim, n_comp, mean_var, seed=0, dtype="f32"):
    X, _ = gaussian_mixture(n, dim, n_comp, mean_var, seed)
    return euclidean_from_points(X, dtype=dtype)
