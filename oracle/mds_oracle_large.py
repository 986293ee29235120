"""Row-blocked FP64 oracle for large n (TEST INFRASTRUCTURE ONLY).

Same method and readings as ``mds_oracle.rand_mds``; the only difference is
memory: at n = 1e5 the Gram matrix would take 80 GB in float64, so every
product G X is taken one block of rows at a time, each block of G being
formed from the matching rows of D with the centring equation of Sec. 6.2,
step 1.  Every entry y_ik = sum_j gamma_ij x_jk is still one library matmul
over the full j range; nothing else is reordered.  Uses plain PyTorch CPU ops
in float64 (multi-threaded), on a host copy of D.

Pinned against ``mds_oracle.rand_mds`` on small inputs (tests/test_oracle_large.py).
"""
from __future__ import annotations

import numpy as np

from .mds_oracle import omega, normalise_column_signs, FORMS, pass_dtypes


def _torch():
    import torch

    return torch


def centring_stats_blocked(D, block: int = 4096):
    """r_i, c_j (means of d^2 over rows / columns) and m, as in
    ``mds_oracle.centring_stats``, accumulated over row blocks in float64."""
    torch = _torch()
    Dt = torch.as_tensor(D)
    n = Dt.shape[0]
    rsum = torch.zeros(n, dtype=torch.float64)
    csum = torch.zeros(n, dtype=torch.float64)
    for a in range(0, n, block):
        b = min(a + block, n)
        D2 = Dt[a:b].to(torch.float64) ** 2
        rsum[a:b] = D2.sum(dim=1)
        csum += D2.sum(dim=0)
    r = (rsum / n).numpy()
    c = (csum / n).numpy()
    m = float(rsum.sum()) / (n * n)
    return r, c, m


def _round_t(x, dtype):
    torch = _torch()
    if dtype == "fp8blk":  # row block of G: its 256 x 256 tiles are whole
        from .mds_oracle import fp8_operand

        return torch.from_numpy(fp8_operand(x.numpy()))
    if dtype == "f64":
        return x
    if dtype == "f32":
        return x.to(torch.float32).to(torch.float64)
    if dtype == "bf16":
        return x.to(torch.float32).to(torch.bfloat16).to(torch.float64)
    if dtype == "bf16x2":  # first two terms of the bfloat16 expansion of the float32 value
        f = x.to(torch.float32)
        b0 = f.to(torch.bfloat16).to(torch.float32)
        b1 = (f - b0).to(torch.bfloat16).to(torch.float32)
        return b0.to(torch.float64) + b1.to(torch.float64)
    raise ValueError(dtype)


def gram_apply_blocked(D, stats, X, gdtype="f64", block: int = 2048):
    """Y = G X with G from D (gamma_ij = -1/2 (d_ij^2 - c_j - r_i + m)), the
    entries of G rounded to ``gdtype`` (storage of the form)."""
    torch = _torch()
    Dt = torch.as_tensor(D)
    r, c, m = stats
    rt = torch.as_tensor(r, dtype=torch.float64)
    ct = torch.as_tensor(c, dtype=torch.float64)
    Xt = torch.as_tensor(X, dtype=torch.float64)
    n = Dt.shape[0]
    Y = torch.empty((n, Xt.shape[1]), dtype=torch.float64)
    if gdtype == "fp8blk" and block % 256:
        raise ValueError("fp8 blocks need row blocks that are multiples of 256")
    for a in range(0, n, block):
        b = min(a + block, n)
        G = -0.5 * (Dt[a:b].to(torch.float64) ** 2 - ct[None, :] - rt[a:b, None] + m)
        Y[a:b] = _round_t(G, gdtype) @ Xt
    return Y.numpy()


def rand_mds_blocked(D, k: int, p: int, q: int, seed: int, form: str = "fp64", block: int = 2048,
                     progress=None):
    """Randomized classical MDS (steps of ``mds_oracle.rand_mds``) with the
    products by G taken block-row-wise.  ``progress(msg)`` is called after
    every pass."""
    n = D.shape[0]
    l = k + p
    if not (1 <= k and p >= 0 and l <= n and q >= 0):
        raise ValueError("need 1 <= k, p >= 0, k + p <= n, q >= 0")
    say = progress or (lambda msg: None)
    stats = centring_stats_blocked(D)
    say("centring statistics done")
    gp, xp = FORMS[form]["proj"]
    from .mds_oracle import round_to, orthonormal_basis

    Q = omega(seed, n, l)
    for it in range(2 * q + 1):  # Omega, then q times two applications (G^T = G)
        gr, xr = pass_dtypes(form, it, q)
        Y = gram_apply_blocked(D, stats, round_to(Q, xr), gr, block)
        Q = orthonormal_basis(Y)
        say(f"range pass {it + 1} done")
    Y = gram_apply_blocked(D, stats, round_to(Q, xp), gp, block)
    B = Q.T @ Y
    B = 0.5 * (B + B.T)
    w, V = np.linalg.eigh(B)
    order = np.argsort(-w, kind="stable")
    theta, V = w[order], V[:, order]
    X = Q @ V[:, :k] * np.sqrt(np.maximum(theta[:k], 0.0))[None, :]
    say("projection and eigensolve done")
    return {"eigvals": theta[:k].copy(), "theta": theta, "coords": normalise_column_signs(X), "Q": Q,
            "stats": stats}
