"""Helpers for the GPU parity tests (comparison only; no method arithmetic)."""
from __future__ import annotations

import sys

import numpy as np
import scipy.linalg


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bf16_round(x: np.ndarray) -> np.ndarray:
    """float64 -> float32 (RNE) -> bfloat16 (RNE), returned as float32."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (r.astype(np.uint32) << 16).view(np.float32)


def rel_eig_err(got, want, floor_rel=1e-12):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    floor = floor_rel * np.max(np.abs(want))
    return np.max(np.abs(got - want) / np.maximum(np.abs(want), floor))


def procrustes_err(X, Xref):
    """Relative Frobenius distance after the best orthogonal alignment."""
    R, _ = scipy.linalg.orthogonal_procrustes(X, Xref)
    return np.linalg.norm(X @ R - Xref) / max(np.linalg.norm(Xref), 1e-300)


def sign_aligned_err(X, Xref):
    s = np.sign(np.sum(X * Xref, axis=0))
    s[s == 0] = 1
    return np.linalg.norm(X * s - Xref) / max(np.linalg.norm(Xref), 1e-300)


def span_cos_min(Q, Qref):
    """Smallest cosine of the principal angles between two orthonormal bases."""
    return float(np.min(np.linalg.svd(Q.T @ Qref, compute_uv=False)))
