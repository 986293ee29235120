#!/usr/bin/env python
"""Benchmark: paper-scale random-projection classical MDS on one MI355X.

Workload: synthetic amplicon reads standing in for the Lake Geneva rbcL
sample of the paper (200 random references of length 400, n = 100,000
reads with 1-5 % substitutions; D = Hamming / 400 in fp32, 40 GB, generated
on the GPU), k = 100 axes, oversample 20, q = 2 power iterations.

A step is one complete run of the method through the C ABI with D resident
in HBM: centring, test matrix, 2q+1 orthonormalised range passes, the
projection pass, the small eigensolve and the coordinates.  The headline
value is the BF16 form's time per MDS; the FP32 form is timed beside it, an
FP64-form run is the accuracy reference, and the FP64 CPU oracle is timed on
a bounded sample.

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "n=1e5 k=100 MDS time & MFMA util, BF16 vs FP32 @1e-3 eig err; p99 latency"

# HBM bytes per launch of the G-pass kernels, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE scaled by a plain copy of known size (profiles/
# mds_n100000_amplicon_k100_bf16_fp32_profile.md), on the n = 1e5, l_pad = 128
# workload.  Valid only while the kernel source is the one measured: the
# sha256 prefix of the file is checked and `traffic` is null otherwise.
TRAFFIC = {
    # range pass over the stored bf16 G; FETCH_SIZE at split-K 3, WRITE_SIZE
    # (split-K partials) at split-K 8: the autotuner chose those in the two runs
    "gpass": {"source": "paper_1803_02272_amd/csrc/k_gpass.hip", "sha256_16": "27b651db8e41ac0e",
              "n": 100000, "l_pad": 128, "form": "bf16", "fetch_gb": 23.064, "write_gb": 0.446},
    # symmetric fp32 projection as three-term bf16 split (k_gpass_x3d), split-K 16 / 12
    "gpass_ref": {"source": "paper_1803_02272_amd/csrc/k_gpass.hip", "sha256_16": "27b651db8e41ac0e",
                  "n": 100000, "l_pad": 128, "form": "bf16", "fetch_gb": 23.765, "write_gb": 0.337},
}

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3, "fp64": 78.6}


def measured_traffic(name, n, l_pad, form):
    """HBM bytes per launch measured for this kernel, workload and source, or None."""
    import hashlib

    t = TRAFFIC.get(name)
    if not t or (t["n"], t["l_pad"], t["form"]) != (n, l_pad, form):
        return None
    with open(os.path.join(ROOT, t["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != t["sha256_16"]:
            return None
    return (t["fetch_gb"] + t["write_gb"]) * 1e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(p / 100.0 * (len(xs) - 1)))))
    return xs[i]


def time_form(mds, torch, D, n, k, p, q, form, steps, warmup, autotune=True):
    # "fp32s": the fp32 form with every pass as the three-term bf16 split
    plan = mds.Plan(n, k, p, q, 0, form="fp32" if form == "fp32s" else form, split_fp32=form == "fp32s")
    tuned = None
    if autotune:
        t0 = time.perf_counter()
        tuned = plan.autotune(D)
        log(f"[bench] form={form}: autotuned splits {tuned} in {time.perf_counter() - t0:.1f} s")
    plan.attach_workspace()
    coords = torch.empty((n, k), dtype=torch.float64, device="cuda")
    eig = torch.empty((k,), dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        plan.run(D, coords, eig)
    torch.cuda.synchronize()
    plan.set_timing(True)
    stream = torch.cuda.current_stream()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        starts[s].record(stream)
        plan.run(D, coords, eig)
        ends[s].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    per_step = [a.elapsed_time(b) for a, b in zip(starts, ends)]
    phases = plan.timings()
    plan.set_timing(False)
    info = plan.info()
    out = {
        "ms": sum(per_step) / len(per_step),
        "wall_ms": wall,
        "p50_ms": percentile(per_step, 50),
        "p99_ms": percentile(per_step, 99),
        "phases": {name: {"count": c, "avg_ms": (t / c if c else 0.0), "total_ms": t / max(steps, 1)}
                   for name, (c, t, _mn, _mx) in phases.items()},
        "eig": eig.double().cpu().numpy(),
        "info": info,
        "gpass_split": info["gpass_split"],
        "autotune": tuned,
    }
    plan.close()
    del coords
    torch.cuda.empty_cache()
    return out


def copy_probe(torch, mib, reps):
    """Plain copy of a known size: reads and writes mib MiB per launch."""
    nb = mib << 20
    src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    print(json.dumps({"copy_probe_bytes_read": nb, "copy_probe_bytes_written": nb, "launches": reps + 1,
                      "ms": ms, "gbs_read_plus_write": 2 * nb / (ms * 1e-3) / 1e9}), flush=True)


def serving_bench(mds, torch, wgpu, seconds, warmup_s, rate, pool_size, budget_gb, slots, seed=0):
    """Serving mix: Poisson arrivals of MDS jobs with n log-uniform in
    [500, 30000], half Gaussian-mixture (50 dims, 10 components, means
    N(0, 25 I)) and half amplicon-Hamming (50 references) distance matrices
    drawn from a device-resident pool, k=20, oversample 10, q=2, BF16 form,
    admitted by the server under an HBM budget.  Latency is submit ->
    completion as observed by the server; requests submitted during the
    warm-up are excluded."""
    import numpy as np

    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(np.log(500), np.log(30000), pool_size))).astype(int)
    pool = []
    t0 = time.perf_counter()
    for i, n in enumerate(ns):
        if i % 2 == 0:
            D = wgpu.mixture_distances(int(n), 50, 10, 25.0, seed=1000 + i)
        else:
            D = wgpu.amplicon_distances(int(n), 50, seed=1000 + i)
        pool.append((mds.Plan(int(n), 20, 10, 2, seed=i, form="bf16"), D))
    torch.cuda.synchronize()
    pool_gb = sum(D.numel() * 4 for _, D in pool) / 1e9
    log(f"[serve] pool of {pool_size} D ({pool_gb:.1f} GB) ready in {time.perf_counter() - t0:.1f} s")
    budget = int(budget_gb * (1 << 30))
    out = {"pool": pool_size, "pool_gb": pool_gb, "budget_gib": budget_gb, "slots": slots, "rate_per_s": rate,
           "seconds": seconds, "warmup_s": warmup_s}
    with mds.Server(budget, slots=slots) as srv:
        t0 = time.perf_counter()
        out["batching_small_n_max"] = srv.autotune(form="bf16", k=20, oversample=10, q=2)
        log(f"[serve] autotuned batching threshold n <= {out['batching_small_n_max']} "
            f"in {time.perf_counter() - t0:.1f} s")
        # saturation: the whole pool submitted at once
        t0 = time.perf_counter()
        tickets = [srv.submit(pl, D)[0] for pl, D in pool]
        for t in tickets:
            assert srv.wait(t)[0] == 0
        burst_s = time.perf_counter() - t0
        out["burst_solves_per_s"] = pool_size / burst_s
        # open loop: Poisson arrivals
        gaps = rng.exponential(1.0 / rate, int(rate * (seconds + warmup_s) * 2) + 16)
        arrivals = np.cumsum(gaps)
        arrivals = arrivals[arrivals < seconds + warmup_s]
        picks = rng.integers(0, pool_size, len(arrivals))
        sub = []
        start = time.perf_counter()
        for a, j in zip(arrivals, picks):
            now = time.perf_counter() - start
            if a > now:
                time.sleep(a - now)
            pl, D = pool[j]
            sub.append((a, j, srv.submit(pl, D)[0]))
        lat, done_at = [], []
        for a, j, t in sub:
            st, tm = srv.wait(t)
            assert st == 0, st
            if a >= warmup_s:
                lat.append(tm["latency_ms"])
                done_at.append(a + tm["latency_ms"] * 1e-3)
        info = srv.stats()
    n_req = len(lat)
    window = max(done_at) - warmup_s if done_at else float("nan")
    out.update({"requests": n_req, "solves_per_s": n_req / window if n_req else None,
                "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99), "max_ms": max(lat) if lat else None,
                "peak_arena_gib": info["peak_bytes"] / (1 << 30), "batched_launches": info["batches"]})
    del pool
    torch.cuda.empty_cache()
    return out


def cpu_baseline(n_full, k, p, q, n_sample, refs):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload;
    time scaled by (n_full / n_sample)^2 (every pass is O(n^2 l))."""
    import numpy as np

    import oracle
    import workloads

    try:
        from threadpoolctl import threadpool_info

        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    reads, _ = workloads.amplicon_reads(n_sample, refs, seed=0)
    D = workloads.hamming_distances(reads)
    t0 = time.perf_counter()
    res = oracle.rand_mds(D, k, p, q, 0)
    dt = time.perf_counter() - t0
    del res, D
    return {
        "value": dt * 1e3 * (n_full / n_sample) ** 2,
        "unit": "ms",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"FP64 numpy oracle (randomized MDS, same k/p/q) on the amplicon recipe at n={n_sample} "
                   f"({refs} refs): {dt:.2f} s measured, scaled by (n/n_sample)^2 to n={n_full}"),
        "measured_s": dt,
        "n_sample": n_sample,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=100000)
    ap.add_argument("--refs", type=int, default=200)
    ap.add_argument("--k", type=int, default=100)
    ap.add_argument("--oversample", type=int, default=20)
    ap.add_argument("--q", type=int, default=2)
    ap.add_argument("--forms", default="bf16,fp32,fp32s,fp64",
                    help="fp32s = the fp32 form with every pass as the three-term bf16 split")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default split-K of every pass")
    ap.add_argument("--cpu-sample", type=int, default=20000)
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="open-loop duration of the serving mix after its warm-up (0 = skip serving)")
    ap.add_argument("--serve-warmup", type=float, default=2.0)
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-pool", type=int, default=64)
    ap.add_argument("--serve-budget-gib", type=float, default=200.0)
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only time a plain device-to-device copy of MIB MiB (stream bandwidth, and the "
                         "known-size reference for the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is a design "
                                   "(row panels over RCCL) and is not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_probe:
        copy_probe(torch, args.copy_probe, max(args.steps, 1))
        return

    import paper_1803_02272_amd as mds
    from workloads import gpu as wgpu

    n, k, p, q = args.n, args.k, args.oversample, args.q
    l = k + p
    log(f"[bench] generating amplicon D n={n} refs={args.refs} on the GPU")
    t0 = time.perf_counter()
    D = wgpu.amplicon_distances(n, args.refs, seed=0)
    log(f"[bench] D ready in {time.perf_counter() - t0:.1f} s")

    forms = [f for f in args.forms.split(",") if f]
    res = {}
    for form in forms:
        steps = args.steps if form != "fp64" else 1
        warm = args.warmup if form != "fp64" else 0
        log(f"[bench] form={form} warmup={warm} steps={steps}")
        res[form] = time_form(mds, torch, D, n, k, p, q, form, steps, warm, autotune=not args.no_autotune)
        log(f"[bench] form={form}: {res[form]['ms']:.2f} ms/step; phases "
            + ", ".join(f"{a}={b['total_ms']:.2f}" for a, b in res[form]["phases"].items() if b["count"]))
    del D
    torch.cuda.empty_cache()

    head = res["bf16"] if "bf16" in res else res[forms[0]]
    head_form = "bf16" if "bf16" in res else forms[0]
    ref_eig = res["fp64"]["eig"] if "fp64" in res else None

    def eig_err(form):
        if ref_eig is None or form not in res:
            return None
        e = res[form]["eig"]
        return float(np.max(np.abs(e - ref_eig) / np.abs(ref_eig)))

    # dominant kernel of the headline form and its roofline.  Algorithmic work:
    # a range pass reads G once (stored bf16 / fp8 G, else the fp32 D it
    # recentres) and does 2 n^2 l flops; the symmetric projection reads the
    # upper triangle of D (n^2 / 2 fp32) and does n^2 l useful flops, which the
    # bf16 and fp8 forms execute as six bf16 products per entry (three-term
    # split of the fp32 operands) on bf16 MFMA.
    flops_pass = 2.0 * n * n * l
    d_bytes = 4  # D is fp32 in this workload
    g_bytes = {"bf16": 2, "fp8": 1}
    x_bytes = {"bf16": 2, "fp8": 2, "fp32": 4, "fp32s": 6, "fp64": 8}
    gb = {"bf16": 2, "fp8": 1, "fp32": 4, "fp32s": 4, "fp64": 8}

    def range_bytes(form):
        return n * n * g_bytes.get(form, d_bytes) + n * l * (x_bytes[form] + 4)

    def mfma_dtype(form):
        # fp8 codes are decoded into bf16 MFMA operands; split passes run on bf16 MFMA
        return "bf16" if form in ("fp8", "fp32s") else form

    def split_proj(form):
        return form in ("bf16", "fp8", "fp32s")

    def range_executed(form):
        """executed MFMA flops of one range pass (six products per entry when split)"""
        return 6.0 * flops_pass if form == "fp32s" else flops_pass

    proj_flops = 1.0 * n * n * l
    proj_bytes = n * n // 2 * d_bytes + n * l * (6 + 4)

    def proj_mfma(form):
        """(executed MFMA flops of one projection, dtype whose peak bounds it)"""
        return (6.0 * proj_flops, "bf16") if split_proj(form) else (proj_flops, form)

    ph = head["phases"]
    cands = {}
    if ph["gpass"]["count"]:
        cands["gpass"] = dict(
            kernel=f"k_gpass<{head_form}> (range pass Y = G X)", total=ph["gpass"]["total_ms"],
            avg=ph["gpass"]["avg_ms"], bytes=range_bytes(head_form), flops=flops_pass,
            bound="hbm" if flops_pass / range_bytes(head_form) < PEAK_TFLOPS[mfma_dtype(head_form)] * 1e12 / (PEAK_HBM_GBS * 1e9)
            else "mfma",
            dtype=mfma_dtype(head_form))
    if ph["gpass_ref"]["count"]:
        pf, pdt = proj_mfma(head_form)
        cands["gpass_ref"] = dict(
            kernel=("k_gpass_x3d (projection, fp32 as 3-term bf16 split, symmetric)" if split_proj(head_form)
                    else f"k_gpass<{head_form}> (projection, symmetric)"),
            total=ph["gpass_ref"]["total_ms"], avg=ph["gpass_ref"]["avg_ms"], bytes=proj_bytes, flops=pf,
            bound="mfma", dtype=pdt)
    for name, unit_bytes in (("write", n * n * (4 + gb[head_form] + (4 if head_form == "bf16" else 0))),
                             ("stats", n * n * 4)):
        if ph[name]["count"]:
            cands[name] = dict(kernel=f"centring {name}", total=ph[name]["total_ms"], avg=ph[name]["avg_ms"],
                               bytes=unit_bytes, flops=0.0, bound="hbm", dtype=head_form)
    dom_name = max(cands, key=lambda c: cands[c]["total"])
    dom = cands[dom_name]
    if dom["bound"] == "hbm":
        achieved = dom["bytes"] / (dom["avg"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    else:
        achieved = dom["flops"] / (dom["avg"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[dom["dtype"]], "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dom_name, n, (l + 15) // 16 * 16, head_form)
    roof["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    roof["kernel"] = dom["kernel"]
    roof["avg_launch_ms"] = dom["avg"]
    roof["algorithmic_bytes_per_launch"] = dom["bytes"]
    roof["algorithmic_flops_per_launch"] = dom["flops"]

    # MFMA utilisation of the G-passes of each form: algorithmic TFLOP/s, and
    # the executed MFMA work over the peak of the dtype it runs on
    gemm = {}
    for form, r in res.items():
        g = r["phases"]["gpass"]
        gr = r["phases"]["gpass_ref"]
        entry = {}
        if g["count"]:
            tf = flops_pass / (g["avg_ms"] * 1e-3) / 1e12
            entry["range_pass_ms"] = g["avg_ms"]
            entry["range_pass_tflops"] = tf
            entry["range_pass_mfma_frac"] = (range_executed(form) / (g["avg_ms"] * 1e-3) / 1e12
                                             / PEAK_TFLOPS[mfma_dtype(form)])
            entry["range_pass_hbm_gbs"] = range_bytes(form) / (g["avg_ms"] * 1e-3) / 1e9
        if gr["count"]:
            pf, pdt = proj_mfma(form)
            entry["proj_pass_ms"] = gr["avg_ms"]
            entry["proj_pass_tflops"] = proj_flops / (gr["avg_ms"] * 1e-3) / 1e12
            entry["proj_pass_mfma"] = "bf16 (six products of three-term splits)" if split_proj(form) else form
            entry["proj_pass_mfma_frac"] = pf / (gr["avg_ms"] * 1e-3) / 1e12 / PEAK_TFLOPS[pdt]
            entry["proj_pass_hbm_gbs"] = proj_bytes / (gr["avg_ms"] * 1e-3) / 1e9
        tot = (g["total_ms"] + gr["total_ms"])
        alg = (2 * q + 1) * flops_pass + proj_flops
        entry["all_passes_tflops"] = alg / (tot * 1e-3) / 1e12 if tot else None
        gemm[form] = entry

    line = {
        "metric": METRIC,
        "value": head["ms"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head_form,
        "data": "synthetic: amplicon reads (random ACGT references, 1-5% substitutions), D = Hamming/400 fp32, "
                "generated on the GPU; stands in for the paper's Lake Geneva rbcL sample",
        "config": {"workload": f"amplicon MDS n={n} refs={args.refs} k={k} oversample={p} q={q}",
                   "n": n, "k": k, "oversample": p, "q": q, "form": head_form},
        "p50_ms": head["p50_ms"],
        "p99_ms": head["p99_ms"],
        "forms": {f: {"ms": r["ms"], "p99_ms": r["p99_ms"], "eig_rel_err_vs_fp64_form": eig_err(f),
                      "phases_ms": {a: round(b["total_ms"], 4) for a, b in r["phases"].items() if b["count"]},
                      "gpass_split": r["gpass_split"], "autotune": r["autotune"],
                      "orth_fallbacks": r["info"]["orth_fallbacks"],
                      "jacobi_sweeps": r["info"]["jacobi_sweeps"]} for f, r in res.items()},
        "gemm": gemm,
        "speedup_bf16_vs_fp32": (res["fp32"]["ms"] / res["bf16"]["ms"]) if ("bf16" in res and "fp32" in res)
        else None,
        "roofline": roof,
    }
    if args.serve_seconds > 0:
        log(f"[bench] serving mix: {args.serve_rate}/s for {args.serve_seconds} s")
        line["serving"] = serving_bench(mds, torch, wgpu, args.serve_seconds, args.serve_warmup, args.serve_rate,
                                        args.serve_pool, args.serve_budget_gib, args.serve_slots)
        log(f"[bench] serving: {line['serving']}")
        line["p99_ms_serving"] = line["serving"]["p99_ms"]
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline: oracle at n={args.cpu_sample}")
        line["cpu_baseline"] = cpu_baseline(n, k, p, q, args.cpu_sample, args.refs)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
