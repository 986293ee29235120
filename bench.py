#!/usr/bin/env python
"""Benchmark: paper-scale random-projection classical MDS on one MI355X.

Workload: synthetic amplicon reads standing in for the Lake Geneva rbcL
sample of the paper (200 random references of length 400, n = 100,000
reads with 1-5 % substitutions; D = Hamming / 400 in fp32, 40 GB, generated
by the library's own distance kernel), k = 100 axes, oversample 20, q = 2
power iterations.

A step is one complete run of the method through the C ABI with D resident
in HBM: centring, test matrix, 2q+1 orthonormalised range passes, the
projection pass, the small eigensolve and the coordinates.  The headline
value is the BF16 form's time per MDS; the FP32 form is timed beside it, an
FP64-form run is the accuracy reference, and the FP64 CPU oracle is timed on
a bounded sample.  The distance kernel that writes D and the threshold-graph
components on the same D are timed once each beside the MDS step.

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

# HBM bytes per launch of the pass kernels, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE scaled by a plain copy of known size (profiles/
# mds_n100000_amplicon_k100_bf16_fp32s_profile.md), on the n = 1e5, l_pad = 128
# workload, bf16 form.  Valid only while the kernel source is the one
# measured: the sha256 prefix of the file is checked and `traffic` is null
# otherwise.
_KS = {"source": "paper_1803_02272_amd/csrc/k_split.hip", "sha256_16": "0adb9b680e01cd0c",
       "n": 100000, "l_pad": 128, "form": "bf16"}
TRAFFIC = {
    # fused centring write + 16-bit range pass 1 (k_split<kWrite, 2 + 2 terms>)
    "write": dict(_KS, fetch_gb=41.550, write_gb=20.935),
    # 16-bit last range pass from D (k_split<kFull, 2 + 1 terms>)
    "gpass_f32": dict(_KS, fetch_gb=41.377, write_gb=0.630),
    # 16-bit symmetric projection (k_split<kSym, 2 + 2 terms>)
    "gpass_ref": dict(_KS, fetch_gb=22.098, write_gb=0.652),
    # range pass over the stored bf16 G (k_gstream)
    "gpass": {"source": "paper_1803_02272_amd/csrc/k_gstream.hip", "sha256_16": "bd7252c166b46630",
              "n": 100000, "l_pad": 128, "form": "bf16", "fetch_gb": 20.587, "write_gb": 0.155},
}

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3, "fp64": 78.6}
PEAK_FP4_TFLOPS = 10100.0
PEAK_FP64_VECTOR_TOPS = 39.3216  # Tops/s of non-fused fp64 vector ops: 256 CUs x 64 lanes x 2.4 GHz


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


# Benchmark variants: name -> Plan keyword arguments.  "bf16" and "fp8" are
# the library's default schedules (16-bit first and last range pass and
# projection: two-term bf16 split of G, of X too except in the last range
# pass, which rounds X to bf16); "bf16a" and "fp8a" run every range pass
# on the stored G (MDS_FLAG_LOWP_ALL_RANGE); "fp32s" is the fp32 form with
# every pass as the three-term bf16 split.
VARIANTS = {
    "bf16": dict(form="bf16"), "bf16a": dict(form="bf16", lowp_all_range=True),
    "fp8": dict(form="fp8"), "fp8a": dict(form="fp8", lowp_all_range=True),
    "fp32": dict(form="fp32"), "fp32s": dict(form="fp32", split_fp32=True), "fp64": dict(form="fp64"),
}


def time_form(mds, torch, D, n, k, p, q, form, steps, warmup, autotune=True):
    plan = mds.Plan(n, k, p, q, 0, **VARIANTS[form])
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
        "steps": steps,
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


def burst_bench(mds, torch, wgpu, jobs, n_lo, n_hi, budget_gb, slots, max_batch, seed=1):
    """Small-job burst: `jobs` MDS jobs with n log-uniform in [n_lo, n_hi]
    (half Gaussian-mixture, half amplicon, k=20, oversample 10, q=2, BF16
    form) submitted at once, served with batching of small jobs (one
    persistent batched launch per group of up to max_batch) and without it.
    Reports solves/s and p50/p99 latency of each."""
    import numpy as np

    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), jobs))).astype(int)
    work = []
    for i, n in enumerate(ns):
        D = (wgpu.mixture_distances(int(n), 50, 10, 25.0, seed=5000 + i) if i % 2 == 0
             else wgpu.amplicon_distances(int(n), 50, seed=5000 + i))
        work.append((mds.Plan(int(n), 20, 10, 2, seed=i, form="bf16"), D))
    torch.cuda.synchronize()
    out = {"jobs": jobs, "n_range": [n_lo, n_hi], "slots": slots, "max_batch": max_batch}
    for label, small_n_max in (("batched", n_hi), ("unbatched", 0)):
        with mds.Server(int(budget_gb * (1 << 30)), slots=slots, small_n_max=small_n_max,
                        max_batch=max_batch) as srv:
            for rep in range(2):  # the first round warms up kernels and the arena
                t0 = time.perf_counter()
                tickets = [srv.submit(pl, D)[0] for pl, D in work]
                lat = []
                for t in tickets:
                    st, tm = srv.wait(t)
                    assert st == 0, st
                    lat.append(tm["latency_ms"])
                wall = time.perf_counter() - t0
            info = srv.stats()
        out[label] = {"solves_per_s": jobs / wall, "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
                      "batched_launches": info["batches"] // 2}
        log(f"[burst] {label}: {out[label]}")
    del work
    torch.cuda.empty_cache()
    return out


def _event_ms(torch, fn, reps=3):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def time_distances(mds, torch, codes, D):
    """mds_hamming_distances writing the benchmark's D: n^2 fp32 entries
    written, 2 n^2 (4 L) fp4 MFMA operations (one-hot inner products)."""
    n, L = codes.shape
    ms = _event_ms(torch, lambda: mds.hamming_distances(codes, out=D))
    wbytes, ops = 4.0 * n * n, 2.0 * n * n * 4 * L
    return {"kernel": "k_hamming (fp4 one-hot, scaled MFMA 16x16x128, D written in fp32)", "ms": ms, "n": n,
            "length": L, "write_gbs": wbytes / ms / 1e6, "hbm_frac": wbytes / ms / 1e6 / PEAK_HBM_GBS,
            "fp4_tflops": ops / ms / 1e9, "fp4_frac": ops / ms / 1e9 / PEAK_FP4_TFLOPS}


def time_euclidean(mds, torch, D, dim, comps, var):
    """mds_euclidean_distances at the low-precision stress shape (n points of
    a Gaussian mixture in dim dimensions), written into D's memory: n^2 fp32
    entries written; 3 n^2 dim / 2 fp64 vector operations over the tiles on
    and above the diagonal (a subtraction, a square and an add per
    coordinate, no fused multiply-add), against the non-fused fp64 vector
    rate of 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 Tops/s."""
    from workloads import gaussian_mixture

    n = D.shape[0]
    X, _ = gaussian_mixture(n, dim, comps, var, seed=0)
    xt = torch.from_numpy(X).cuda()
    ms = _event_ms(torch, lambda: mds.euclidean_distances(xt, out=D))
    del xt
    wbytes, ops = 4.0 * n * n, 1.5 * n * n * dim
    return {"kernel": "k_euclid (64 x 64 tiles on and above the diagonal, fp64 vector, D written in fp32)",
            "ms": ms, "n": n, "dim": dim, "write_gbs": wbytes / ms / 1e6, "hbm_frac": wbytes / ms / 1e6 / PEAK_HBM_GBS,
            "fp64_vector_tops": ops / ms / 1e9, "alu_frac": ops / ms / 1e9 / PEAK_FP64_VECTOR_TOPS}


def time_components(mds, torch, D, theta):
    """mds_threshold_components over the upper triangle of D: 2 n (n - 1)
    bytes of fp32 entries read."""
    n = D.shape[0]
    out = {}
    ms = _event_ms(torch, lambda: out.update(r=mds.threshold_components(D, theta)))
    nbytes = 2.0 * n * (n - 1)
    return {"kernel": "k_cc_tiles (LDS + global union-find over the upper triangle)", "ms": ms,
            "threshold": theta, "components": int(out["r"][1].item()), "read_gbs": nbytes / ms / 1e6,
            "hbm_frac": nbytes / ms / 1e6 / PEAK_HBM_GBS}


def cpu_baseline(D, n, k, p, q, sample_rows):
    """The FP64 row-blocked oracle, as it stands, on a bounded sample of the
    benchmark workload itself (n = the benchmark's n, the same D copied to
    the host): the centring statistics over all of D, the test matrix, one
    orthonormalisation and one product G X over `sample_rows` rows of D are
    timed; the estimate adds up the method's 2q + 2 products (each row block
    of a product costs the same at fixed n, so the sample scales linearly in
    rows), 2q + 1 orthonormalisations and the rest as measured."""
    import numpy as np

    import oracle
    from oracle import mds_oracle_large as OL

    try:
        from threadpoolctl import threadpool_info

        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    import torch

    threads = max(threads, torch.get_num_threads())
    l = k + p
    t0 = time.perf_counter()
    Dh = D.cpu().numpy()
    copy_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    stats = OL.centring_stats_blocked(Dh)
    t_stats = time.perf_counter() - t0
    t0 = time.perf_counter()
    X = oracle.omega(0, n, l)
    t_omega = time.perf_counter() - t0
    t0 = time.perf_counter()
    Q = oracle.orthonormal_basis(X)
    t_orth = time.perf_counter() - t0
    rows = min(sample_rows, n)
    t0 = time.perf_counter()
    Y = OL.gram_apply_blocked(Dh[:rows], stats, Q)
    t_rows = time.perf_counter() - t0
    assert Y.shape == (rows, l) and np.all(np.isfinite(Y))
    del Dh, Y, Q, X
    t_pass = t_rows * n / rows
    est = t_stats + t_omega + (2 * q + 2) * t_pass + (2 * q + 1) * t_orth
    measured = t_stats + t_omega + t_orth + t_rows
    return {
        "value": est * 1e3,
        "unit": "ms",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"FP64 row-blocked oracle at n={n} on this D: centring statistics over all of D "
                   f"({t_stats:.1f} s), Omega ({t_omega:.1f} s), one Householder QR of n x l ({t_orth:.2f} s) "
                   f"and one product G X over {rows} of the {n} rows ({t_rows:.1f} s) measured; "
                   f"estimate = stats + Omega + {2 * q + 2} products x {n}/{rows} + {2 * q + 1} QR"),
        "measured_s": measured,
        "n": n,
        "sample_rows": rows,
        "d_to_host_s": copy_s,
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
    ap.add_argument("--forms", default="bf16,bf16a,fp32,fp32s,fp64",
                    help="comma list of " + ", ".join(VARIANTS) + " (bf16a/fp8a: every range pass on the "
                         "stored G; fp32s: the fp32 form with every pass as the three-term bf16 split)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default split-K of every pass")
    ap.add_argument("--cpu-sample-rows", type=int, default=2048,
                    help="rows of D over which one oracle product G X is timed for the CPU baseline")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="open-loop duration of the serving mix after its warm-up (0 = skip serving)")
    ap.add_argument("--serve-warmup", type=float, default=5.0)
    ap.add_argument("--burst-jobs", type=int, default=256,
                    help="small-job burst served with and without batching (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-pool", type=int, default=64)
    ap.add_argument("--serve-budget-gib", type=float, default=200.0)
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--euclid-dim", type=int, default=200,
                    help="dimension of the points for the Euclidean distance timing (0: skip)")
    ap.add_argument("--cc-threshold", type=float, default=0.03,
                    help="threshold of the components measurement (distance units)")
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
    from workloads import amplicon_reads

    reads, _ = amplicon_reads(n, args.refs, seed=0)
    codes = torch.from_numpy(reads).cuda()
    D = mds.hamming_distances(codes)
    torch.cuda.synchronize()
    log(f"[bench] D ready in {time.perf_counter() - t0:.1f} s")
    distances = time_distances(mds, torch, codes, D)
    log(f"[bench] hamming distances: {distances}")
    components = time_components(mds, torch, D, args.cc_threshold)
    log(f"[bench] threshold components: {components}")

    forms = [f for f in args.forms.split(",") if f]
    for f in forms:
        if f not in VARIANTS:
            raise SystemExit(f"unknown form {f!r}; choose from {', '.join(VARIANTS)}")
    res = {}
    for form in forms:
        steps = args.steps if form != "fp64" else 1
        warm = args.warmup if form != "fp64" else 0
        log(f"[bench] form={form} warmup={warm} steps={steps}")
        res[form] = time_form(mds, torch, D, n, k, p, q, form, steps, warm, autotune=not args.no_autotune)
        log(f"[bench] form={form}: {res[form]['ms']:.2f} ms/step; phases "
            + ", ".join(f"{a}={b['total_ms']:.2f}" for a, b in res[form]["phases"].items() if b["count"]))

    head_form = "bf16" if "bf16" in res else forms[0]
    head = res[head_form]
    ref_eig = res["fp64"]["eig"] if "fp64" in res else None

    def eig_err(form):
        if ref_eig is None or form not in res:
            return None
        e = res[form]["eig"]
        return float(np.max(np.abs(e - ref_eig) / np.abs(ref_eig)))

    # Algorithmic work of every kernel phase (D is fp32 here; l = k + p, the
    # padded l_pad only in the executed MFMA counts):
    #   stats      reads the tiles of D on and above the diagonal: 2 n^2 bytes
    #   write      fused centring write + first range pass (bf16 form): reads
    #              D (4 n^2), writes the bf16 G (2 n^2); the pass is 16-bit
    #              (two-term split, 3 bf16 products per entry) by default, a
    #              bf16 pass in the bf16a variant
    #   gpass      a range pass over the stored G (bf16 2 n^2 / fp8 n^2 bytes)
    #              or over D recentred on the fly (fp32, fp64 forms: 4 n^2)
    #   gpass_f32  the 16-bit last range pass of the bf16/fp8 forms from D
    #              (4 n^2 bytes, bf16 X, 2 bf16 products per entry; the fp8
    #              form's first range pass, with two-term X and 3 products,
    #              is counted here too)
    #   gpass_ref  the symmetric projection: the upper triangle of D (2 n^2
    #              bytes), n^2 l useful flops (3 bf16 products per entry for
    #              the 16-bit projection of the bf16/fp8 forms, 6 for the
    #              fp32 split of fp32s)
    # plus the tall operand and the fp32 split-K partials per pass
    # (n l (x_bytes + 4)).
    l_pad = (l + 15) // 16 * 16
    x_bytes = {"bf16": 2, "fp8": 2, "fp32": 4, "fp64": 8, "split": 6}

    def split_of(form):
        return form in ("bf16", "bf16a", "fp8", "fp8a", "fp32s")

    def kernel_model(form, phase):
        """(bytes, algorithmic flops, executed MFMA flops, MFMA dtype, label) per launch.  Algorithmic
        flops are the method's (2 n^2 l per range product, n^2 l for the symmetric projection);
        executed MFMA flops count the padded l and every product of a split (3 for two terms, 6 for
        three)."""
        base = VARIANTS[form]["form"]
        lowp = base in ("bf16", "fp8")
        if phase == "stats":
            return 2.0 * n * n, 0.0, 0.0, None, "k_stats (centring statistics, upper-triangle tiles)"
        if phase == "write":
            if form == "bf16":
                return (6.0 * n * n + n * l * (6 + 4), 2.0 * n * n * l, 3 * 2.0 * n * n * l_pad, "bf16",
                        "k_split<kWrite, 2 + 2 terms> (fused centring write + 16-bit range pass 1)")
            if form == "bf16a":
                return (6.0 * n * n + n * l * (2 + 4), 2.0 * n * n * l, 2.0 * n * n * l_pad, "bf16",
                        "k_gpass<bf16, from D> (fused centring write + bf16 range pass 1)")
            return 5.0 * n * n, 0.0, 0.0, None, "k_center_write_fp8"
        if phase == "gpass":
            if lowp:
                gb = 2 if base == "bf16" else 1
                label = "k_gstream (range pass over the stored bf16 G)" if base == "bf16" else \
                    "k_gpass<fp8> (range pass over the stored fp8 G)"
                return (gb * n * n + n * l * (2 + 4), 2.0 * n * n * l, 2.0 * n * n * l_pad, "bf16", label)
            if form == "fp32s":
                return (4.0 * n * n + n * l * (6 + 4), 2.0 * n * n * l, 6 * 2.0 * n * n * l_pad, "bf16",
                        "k_split<kFull, 3 terms> (fp32 range pass as three-term split)")
            return (4.0 * n * n + n * l * (x_bytes[base] + 4 * (2 if base == "fp64" else 1)), 2.0 * n * n * l,
                    2.0 * n * n * l_pad, base, f"k_gpass<{base}, from D> (range pass)")
        if phase == "gpass_f32":
            if base == "bf16":
                return (4.0 * n * n + n * l * (2 + 4), 2.0 * n * n * l, 2 * 2.0 * n * n * l_pad, "bf16",
                        "k_split<kFull, 2 + 1 terms> (16-bit last range pass from D, bf16 X)")
            return (4.0 * n * n + n * l * (4 + 4), 2.0 * n * n * l, 2.5 * 2.0 * n * n * l_pad, "bf16",
                    "k_split<kFull, 2 + 2 / 2 + 1 terms> (16-bit first and last range passes from D)")
        if phase == "gpass_ref":
            if lowp:
                return (2.0 * n * n + n * l * (6 + 4), 1.0 * n * n * l, 3.0 * n * n * l_pad, "bf16",
                        "k_split<kSym, 2 + 2 terms> (16-bit symmetric projection)")
            if form == "fp32s":
                return (2.0 * n * n + n * l * (6 + 4), 1.0 * n * n * l, 6.0 * n * n * l_pad, "bf16",
                        "k_split<kSym, 3 terms> (fp32 symmetric projection as three-term split)")
            return (2.0 * n * n + n * l * (x_bytes[base] + 4 * (2 if base == "fp64" else 1)), 1.0 * n * n * l,
                    1.0 * n * n * l_pad, base, f"k_gpass<{base}> (symmetric projection)")
        return None

    def roof_of(form, phase):
        r = res[form]["phases"][phase]
        m = kernel_model(form, phase)
        if not r["count"] or m is None:
            return None
        nbytes, aflops, xflops, mdt, label = m
        t_hbm = nbytes / (PEAK_HBM_GBS * 1e9)
        t_mfma = xflops / (PEAK_TFLOPS[mdt] * 1e12) if mdt else 0.0
        avg = r["avg_ms"] * 1e-3
        if t_hbm >= t_mfma:
            ach = nbytes / avg / 1e9
            out = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
        else:
            # MFMA-bound: the work the MFMA units execute (padded l, six
            # products per entry for a split pass) against the dtype's peak
            ach = xflops / avg / 1e12
            out = {"bound": "mfma", "achieved": ach, "peak": PEAK_TFLOPS[mdt], "unit": "TFLOP/s"}
        out.update({"frac": out["achieved"] / out["peak"], "kernel": label, "avg_launch_ms": r["avg_ms"],
                    "launches_per_step": r["count"] / max(res[form]["steps"], 1),
                    "algorithmic_bytes_per_launch": nbytes, "algorithmic_flops_per_launch": aflops,
                    "executed_mfma_flops_per_launch": xflops, "mfma_dtype": mdt,
                    "hbm_gbs": nbytes / avg / 1e9,
                    "mfma_frac": (xflops / avg / 1e12 / PEAK_TFLOPS[mdt]) if mdt else None})
        return out

    kernels = {}
    for form in res:
        kernels[form] = {ph: roof_of(form, ph) for ph in ("stats", "write", "gpass", "gpass_f32", "gpass_ref")
                         if roof_of(form, ph) is not None}
    hp = head["phases"]
    dom_name = max(kernels[head_form], key=lambda ph: hp[ph]["total_ms"])
    roof = dict(kernels[head_form][dom_name])
    roof["phase"] = dom_name
    roof["traffic"] = measured_traffic(dom_name, n, l_pad, head_form)
    roof["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"

    # GEMM passes of each form: every pass kernel's time is counted (the
    # fused first pass inside "write" too), against the method's algorithmic
    # flops, (2q + 1) range products 2 n^2 l and the projection's n^2 l
    gemm = {}
    for form, r in res.items():
        ph = r["phases"]
        entry = {}
        for name in ("write", "gpass", "gpass_f32", "gpass_ref"):
            kr = kernels[form].get(name)
            if kr is not None and kr["algorithmic_flops_per_launch"] > 0:
                entry[name] = {"avg_ms": kr["avg_launch_ms"], "launches_per_step": kr["launches_per_step"],
                               "hbm_gbs": kr["hbm_gbs"], "mfma_frac": kr["mfma_frac"], "bound": kr["bound"],
                               "frac": kr["frac"]}
        pass_phases = ["gpass", "gpass_f32", "gpass_ref"] + (["write"] if ph["write"]["count"] and
                                                               kernel_model(form, "write")[1] > 0 else [])
        tot = sum(ph[x]["total_ms"] for x in pass_phases)
        alg = (2 * q + 1) * 2.0 * n * n * l + 1.0 * n * n * l
        entry["pass_phases"] = pass_phases
        entry["passes_ms_per_step"] = tot
        entry["all_passes_tflops"] = alg / (tot * 1e-3) / 1e12 if tot else None
        gemm[form] = entry
    rng_bf16 = kernels.get("bf16", {}).get("gpass")
    mfma_target = {"target_frac": 0.5, "kernel": "bf16 range pass over the stored G",
                   "measured_frac": rng_bf16["mfma_frac"] if rng_bf16 else None,
                   "met": bool(rng_bf16 and rng_bf16["mfma_frac"] >= 0.5),
                   "note": "at 2 bytes of G per 2 l flops the pass is HBM-bound: its MFMA fraction is capped at "
                           f"{2 * l_pad / 2 * PEAK_HBM_GBS * 1e9 / (PEAK_TFLOPS['bf16'] * 1e12):.2f} "
                           "at the HBM peak"}

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
        "kernels": kernels,
        "gemm": gemm,
        "mfma_target": mfma_target,
        "speedup_bf16_vs_fp32": (res["fp32"]["ms"] / res["bf16"]["ms"]) if ("bf16" in res and "fp32" in res)
        else None,
        "roofline": roof,
        "distances": distances,
        "components": components,
    }
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline: row-blocked oracle at n={n}, {args.cpu_sample_rows} sample rows")
        line["cpu_baseline"] = cpu_baseline(D, n, k, p, q, args.cpu_sample_rows)
        log(f"[bench] cpu baseline: {line['cpu_baseline']}")
    else:
        line["cpu_baseline"] = None
    line["distances_euclidean"] = None
    if args.euclid_dim > 0:
        # last use of D's memory (after the MDS runs and the CPU baseline):
        # the Euclidean kernel overwrites it
        line["distances_euclidean"] = time_euclidean(mds, torch, D, args.euclid_dim, 50, 9.0)
        log(f"[bench] euclidean distances: {line['distances_euclidean']}")
    del D
    torch.cuda.empty_cache()
    if args.serve_seconds > 0:
        log(f"[bench] serving mix: {args.serve_rate}/s for {args.serve_seconds} s")
        line["serving"] = serving_bench(mds, torch, wgpu, args.serve_seconds, args.serve_warmup, args.serve_rate,
                                        args.serve_pool, args.serve_budget_gib, args.serve_slots)
        log(f"[bench] serving: {line['serving']}")
        line["p99_ms_serving"] = line["serving"]["p99_ms"]
    if args.burst_jobs > 0:
        # the low end of the serving mix's sizes (batching does not pay there: one workgroup per
        # instance against whole-device plans) and small instances, where it does
        line["serving_burst"] = burst_bench(mds, torch, wgpu, args.burst_jobs, 500, 2048, args.serve_budget_gib,
                                            args.serve_slots, 64)
        log(f"[burst] n 500-2048: {line['serving_burst']}")
        line["serving_burst_small"] = burst_bench(mds, torch, wgpu, 4 * args.burst_jobs, 48, 400,
                                                  args.serve_budget_gib, args.serve_slots, 256)
        log(f"[burst] n 48-400: {line['serving_burst_small']}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
