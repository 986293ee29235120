"""Serving runtime (mds_server_*): continuous batching on one GPU.

Each job in a mixed stream must give exactly the result of the same plan run
alone (bit-identical: same kernels, same launch configuration, deterministic
reductions), while the server overlaps jobs and admits them by memory budget.
"""
import time

import pytest

from gpu_util import procrustes_err, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1803_02272_amd as mds  # noqa: E402
from paper_1803_02272_amd import _capi  # noqa: E402
from workloads import gpu as WG  # noqa: E402


def make_D(kind, n, seed):
    if kind == "gm":
        return WG.mixture_distances(n, 50, 10, 25.0, seed=seed)
    return WG.amplicon_distances(n, 50, seed=seed)


MIX = [  # (kind, n, k, p, q, form)
    ("gm", 517, 20, 10, 2, "bf16"), ("amp", 3001, 20, 10, 2, "bf16"), ("gm", 1200, 20, 10, 2, "fp32"),
    ("amp", 9000, 20, 10, 2, "bf16"), ("gm", 700, 5, 3, 1, "fp64"), ("amp", 4444, 20, 10, 2, "bf16"),
    ("gm", 2500, 30, 10, 2, "bf16"), ("amp", 600, 20, 10, 0, "fp32"), ("gm", 6000, 20, 10, 2, "bf16"),
    ("amp", 1500, 20, 10, 2, "bf16"), ("gm", 15000, 20, 10, 2, "bf16"), ("amp", 800, 12, 4, 3, "fp32"),
]


def alone(plan, D):
    c, e = plan.run(D)
    torch.cuda.synchronize()
    return c.clone(), e.clone()


# batched small jobs agree with the standalone run to the form's rounding
EIG_TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16": 1e-4}


@pytest.mark.parametrize("batching", [False, True])
def test_mix_matches_alone_under_budget(batching):
    jobs = []
    for i, (kind, n, k, p, q, form) in enumerate(MIX):
        D = make_D(kind, n, seed=i)
        jobs.append((mds.Plan(n, k, p, q, seed=100 + i, form=form), D))
    sizes = sorted(pl.workspace_size() for pl, _ in jobs)
    budget = sum(sizes[-3:]) + (1 << 20)  # at most ~3 large jobs resident: forces queueing
    say(f"[serve] {len(jobs)} jobs, budget {budget / 2**20:.0f} MiB, 4 slots, batching {batching}")
    with mds.Server(budget, slots=4, small_n_max=2048 if batching else 0) as srv:
        tickets = [srv.submit(pl, D) for pl, D in jobs]
        results = [srv.wait(t) for t, _, _ in tickets]
        st = srv.stats()
    assert all(r[0] == _capi.OK for r in results), results
    assert st["running"] == 0 and st["queued"] == 0 and st["used_bytes"] == 0
    assert 0 < st["peak_bytes"] <= budget and st["completed"] == len(jobs)
    if not batching:
        assert st["batches"] == 0
    for (pl, D), (t, c, e), (status, times) in zip(jobs, tickets, results):
        ca, ea = alone(pl, D)
        say(f"    n={pl.n} form={pl.form}: latency {times['latency_ms']:.2f} ms (queue {times['queue_ms']:.2f})")
        assert times["latency_ms"] >= times["run_ms"] >= 0
        if batching and pl.n <= 2048:
            rel = (e - ea).abs().max().item() / max(ea.abs().max().item(), 1e-300)
            assert rel < EIG_TOL[pl.form], (pl.n, pl.form, rel)
            assert procrustes_err(c.cpu().numpy(), ca.cpu().numpy()) < 1e-3
            idx = c.abs().argmax(dim=0)
            assert torch.all(c[idx, torch.arange(pl.k, device=c.device)] > 0)
        else:
            assert torch.equal(c, ca) and torch.equal(e, ea), f"n={pl.n} differs from the standalone run"


def test_served_bf16_jobs_against_the_plain_oracle():
    """Served BF16 jobs of the mix (plan path and batched small jobs) against
    the plain FP64 oracle at the form's stated 1e-3 bar."""
    import numpy as np

    import oracle as O
    from gpu_util import rel_eig_err

    picks = [("gm", 517, 1), ("amp", 3001, 2), ("gm", 2500, 3), ("amp", 9000, 4), ("gm", 15000, 5)]
    jobs = [(mds.Plan(n, 20, 10, 2, seed=s, form="bf16"), make_D(kind, n, seed=s)) for kind, n, s in picks]
    say(f"[serve] {len(jobs)} bf16 jobs against the plain oracle")
    with mds.Server(1 << 34, slots=4, small_n_max=1024) as srv:
        tickets = [srv.submit(pl, D) for pl, D in jobs]
        res = [srv.wait(t) for t, _, _ in tickets]
    assert all(r[0] == _capi.OK for r in res)
    for (pl, D), (t, c, e) in zip(jobs, tickets):
        ref = O.rand_mds(D.cpu().numpy(), 20, 10, 2, pl.seed)
        err = rel_eig_err(e.cpu().numpy(), ref["eigvals"])
        say(f"    n={pl.n}: eig rel err vs plain oracle {err:.2e}")
        assert err < 1e-3


def test_cancel_nonfinite_budget_and_tickets():
    import ctypes

    D_big = make_D("amp", 20000, seed=5)
    D_small = make_D("gm", 900, seed=6)
    big = mds.Plan(20000, 20, 10, 2, seed=1, form="bf16")
    small = mds.Plan(900, 20, 10, 2, seed=2, form="bf16")
    nan_D = D_small.clone()
    nan_D[3, 7] = float("nan")
    say("[serve] cancel / non-finite / budget / tickets")
    with mds.Server(big.workspace_size() + 8 * small.workspace_size(), slots=1, small_n_max=0) as srv:
        t0 = srv.submit(big, D_big)[0]
        ts = [srv.submit(small, D_small)[0] for _ in range(3)]
        tn = srv.submit(small, nan_D)[0]
        srv.cancel(ts[-1])  # the big job holds the only slot: this one is still queued
        assert srv.wait(ts[-1])[0] == _capi.ERR_CANCELLED
        with pytest.raises(mds.MdsError) as ei:
            srv.cancel(987654321)
        assert ei.value.status == _capi.ERR_INVALID_ARG
        assert srv.wait(t0)[0] == _capi.OK
        for t in ts[:2]:
            assert srv.wait(t)[0] == _capi.OK
        assert srv.wait(tn)[0] == _capi.ERR_NONFINITE  # only the job with the NaN fails
        with pytest.raises(mds.MdsError):
            srv.poll(t0)  # a terminal status released the ticket
        # once admitted, a job can no longer be cancelled
        t1 = srv.submit(big, D_big)[0]
        t_end = time.time() + 30
        while srv.stats()["queued"]:
            assert time.time() < t_end, "job never admitted"
        with pytest.raises(mds.MdsError) as ei:
            srv.cancel(t1)
        assert ei.value.status == _capi.ERR_STATE
        assert srv.wait(t1)[0] == _capi.OK
        # a job whose workspace exceeds the whole budget is refused at submit,
        # before any of its pointers is used
        huge = mds.Plan(60000, 20, 10, 2, seed=3, form="bf16")
        t = ctypes.c_uint64()
        st = _capi.lib().mds_submit(srv._h, huge.handle, ctypes.c_void_p(D_big.data_ptr()), ctypes.c_void_p(256),
                                    ctypes.c_void_p(256), ctypes.byref(t))
        assert st == _capi.ERR_BUDGET


def test_small_jobs_batched_in_one_launch():
    """A burst of small jobs behind one large job: they queue, then run
    together as batched launches, each within the form's tolerance."""
    probs = [("gm", 300 + 97 * i, 100 + i) for i in range(20)]
    big = mds.Plan(12000, 20, 10, 2, seed=9, form="bf16")
    Dbig = make_D("amp", 12000, seed=9)
    jobs = [(mds.Plan(n, 20, 10, 2, seed=s, form="bf16"), make_D(kind, n, seed=s)) for kind, n, s in probs]
    say(f"[serve] 1 large + {len(jobs)} small jobs, 2 slots")
    with mds.Server(1 << 33, slots=2, small_n_max=4096, max_batch=8) as srv:
        tb = srv.submit(big, Dbig)[0]
        tickets = [srv.submit(pl, D) for pl, D in jobs]
        res = [srv.wait(t) for t, _, _ in tickets]
        assert srv.wait(tb)[0] == _capi.OK
        st = srv.stats()
    assert all(r[0] == _capi.OK for r in res)
    assert st["batches"] >= len(jobs) // 8
    for (pl, D), (t, c, e) in zip(jobs, tickets):
        ca, ea = alone(pl, D)
        rel = (e - ea).abs().max().item() / ea.abs().max().item()
        assert rel < EIG_TOL["bf16"], (pl.n, rel)
