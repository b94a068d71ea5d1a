#!/usr/bin/env python3
"""Benchmark of the fast-SSA hot path on one MI355X.

Workload (one "step" = one pass of the whole hot path over one series):
N = 100000, L = 50000, k = 20 -- five sinusoids + exp(-t/50000) trend +
AR(1) noise (seeded synthetic series; stands in for the long temperature record
of the paper's Sec. 7.1).  A step embeds the series (spectrum), runs the
truncated SVD (Golub-Kahan-Lanczos with full reorthogonalization, FFT
products) and Hankelizes each of the 20 eigentriples into its elementary
series.  The series is resident in HBM before timing starts.

Prints one JSON line:
  value       eigentriples/s over the timed region (k * steps / seconds)
  roofline    the dominant kernel class: algorithmic bytes per launch over its
              HIP-event-measured launch duration (events recorded on the plan's
              stream during the timed region), against 8 TB/s HBM
  cpu_baseline  the FP64 oracle (tier B: Lanczos + direct row products +
              direct antidiagonal averaging) timed on a bounded sample on this
              host and scaled to the same number of steps and triples
  roofline.traffic  HBM bytes per launch of that kernel from two rocprofv3
              counter runs (FETCH_SIZE, WRITE_SIZE; see
              paper_0911_4498_amd/pmc_traffic.py), null unless the summary in
              profiles/ was taken from the current library sources
  served      a bounded served leg: --served-requests (120) requests of the
              served-stream workload below at 100 req/s, p50/p99 latency
With --workload many: the many-series workload instead (4096 series, N uniform
in [2000, 20000], L = N/2, k = 16, seeded), solved together by the batched
engine (ssa_batch_*); the JSON line also reports the single-series path on a
sample of the same series, one series at a time, on the same GPU.
With --workload served: a Poisson stream of requests (N log-uniform in
[1e3, 1e6], L in {N/4, N/2}, k in [8, 32], seeded) at each of --rates;
every request goes to the continuous-batching server (ssa_server_*): N <= --batched-n-max
(8192) to its batched engine, longer ones to its long path (single-series plans bound to
regions of the same pool, --long-slots (4) at a time, one check interval per tick);
reports p50/p99 latency from arrival to complete outputs, and throughput.
With --workload long: the very long series (N = 2^24, L = N/2, k = 50) through
the single-series path with the basis capped by thick restart (--d-max,
--restart-keep); suggested --steps 2 --warmup 1.
--reorth 1 selects one-sided reorthogonalization (single, many, served).
With --workload 2d: 2D-SSA of seeded plane-wave arrays (--s2-sizes), window half the
array, k = 16.
Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--pmc-copy]
                       [--workload single|many|served|hmatrix|realizations|long] [--reorth 0|1]
                       [--series S] [--sample S1] [--rates R1,R2] [--requests Q] [--slots S]
                       [--pool-gb G] [--long-slots S] [--served-requests Q] [--d-max D]
                       [--restart-keep M]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N, L, K_TRIPLES = 100_000, 50_000, 20
# kernel-name substring (as rocprofv3 prints it) of each profiled kernel class
CLASS_KERNEL = {"pass1": "k_pass1<0", "pass2": "k_pass2_matvec", "pass3": "k_pass3<0",
                "cgs_dots": "k_cgs_project", "cgs_reduce": "k_cgs_reduce", "cgs_update": "k_cgs_update",
                "ritz": "k_ritz", "recon_pass1": "k_pass1<2", "recon_pass2": "k_pass2_recon",
                "recon_pass3": "k_pass3<1"}
# on the fused half-step (the default single-series path) passes 1 and 3 carry the update
# and the projection: their kernels are these
CLASS_KERNEL_FUSED = {**CLASS_KERNEL, "pass1": "k_p1_update", "pass3": "k_p3_project"}


def traffic_summary_path(cls, workload="c2"):
    return os.path.join(ROOT, "profiles", f"{workload}_{cls}_traffic.txt")


def traffic_per_launch(cls, workload="c2"):
    """HBM bytes per launch of the class's kernel from the committed counter summary,
    or None if there is none or the library sources changed since it was taken."""
    from paper_0911_4498_amd import pmc_traffic
    s = pmc_traffic.load_summary(traffic_summary_path(cls, workload))
    if not s or s.get("source_sha256") != pmc_traffic.source_hash():
        return None
    return float(s["traffic_bytes_per_launch"])


def copy_calibration():
    """A plain copy of known size (256 MiB read, 256 MiB written) for scaling the
    FETCH_SIZE / WRITE_SIZE counters; only useful under rocprofv3 --pmc."""
    import torch
    n = 64 * 1024 * 1024  # floats
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst


def host_cpu():
    """The host CPU model (from /proc/cpuinfo) and its logical CPU count."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "host_logical_cpus": os.cpu_count()}


def cpu_baseline(f, steps_gpu):
    """Oracle timed on a bounded sample: K_TRIPLES Lanczos steps (2 direct products
    each, OpenMP over rows) and one direct rank-1 Hankelization; scaled to the GPU's
    step count and to K_TRIPLES Hankelizations."""
    import numpy as np

    import oracle
    from paper_0911_4498_amd import inputs
    p0 = inputs.start_vector(L, 4242)
    t0 = time.perf_counter()
    s, U, V, steps, _ = oracle.lanczos_svd(f, L, K_TRIPLES, p0, d_max=K_TRIPLES, check_every=10**6)
    t1 = time.perf_counter()
    t_step = (t1 - t0) / max(steps, 1)
    t2 = time.perf_counter()
    oracle.rank1_hankelize(float(s[0]), U[:, 0], V[:, 0])
    t_hank = time.perf_counter() - t2
    est = steps_gpu * t_step + K_TRIPLES * t_hank
    return {
        "value": K_TRIPLES / est,
        "unit": "eigentriples/s",
        "cores": oracle.num_threads(),
        **host_cpu(),
        "kind": "oracle",
        "sample": (f"tier-B oracle: {steps} Lanczos steps ({2 * steps} direct products, {t_step:.3f} s/step) "
                   f"+ 1 direct rank-1 Hankelization ({t_hank:.2f} s) at N={N}, L={L}; scaled to "
                   f"{steps_gpu} steps and {K_TRIPLES} Hankelizations"),
        "sample_seconds": round(t1 - t0 + t_hank, 2),
    }


def bench_many(args):
    """Many-series workload: batched engine vs one series at a time (eigentriples/s)."""
    import numpy as np
    import torch

    from paper_0911_4498_amd import inputs, ssa
    dev = torch.device("cuda:0")
    ns, k = args.series, 16
    print(f"# generating {ns} series", file=sys.stderr, flush=True)
    host = [inputs.c3_series(s) for s in range(ns)]
    series = [torch.tensor(f, device=dev) for f, _, _ in host]
    Ls = [L for _, _, L in host]
    Ns = np.array([N for _, N, _ in host])
    keys = list(range(ns))
    eng = ssa.Batch(n_max=20000, k_max=k, max_series=ns, reorth=args.reorth)
    steps = []

    def step():
        out = eng.solve(series, Ls, [k] * ns, keys=keys)
        steps.append(out["info"])
        return out

    print(f"# warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    eng.profile_enable()  # every kernel class bracketed by HIP events on the engine's stream
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    prof = eng.profile_read()
    eng.profile_enable(on=False)
    info = steps[-1].cpu().numpy()
    # only the triples of series whose stopping rule held count (equal accuracy)
    n_conv = int(info[:, 1].sum())
    rate_b = n_conv * k * args.steps / t_b
    rate_b_all = ns * k * args.steps / t_b
    for name, (n_l, ms_l) in sorted(prof.items(), key=lambda kv: -kv[1][1]):
        print(f"#   {name:7s} launches={n_l:5d} time={ms_l:9.2f} ms", file=sys.stderr)
    # algorithmic bytes of the Gram-Schmidt launches: a projection against ncols columns reads
    # (ncols + 1) n floats (columns and r), the update (ncols + 1) n and writes n; side 0 runs
    # for j = 1..d+1 with ncols = j-1 over Ki entries, side 1 for j = 1..d with ncols = j over Li
    Li = np.minimum(np.array(Ls), Ns - np.array(Ls) + 1).astype(np.float64)
    Ki = np.maximum(np.array(Ls), Ns - np.array(Ls) + 1).astype(np.float64)
    d = info[:, 0].astype(np.float64)
    # (one-sided: side 0 projects against no columns, 3 Ki floats per launch)
    side0 = 12.0 * Ki * (d + 1) if args.reorth else 4.0 * Ki * (d + 1) * (d + 3)
    cgs_bytes = args.steps * float(np.sum(side0 + 4.0 * Li * d * (d + 4)))
    n_cgs, ms_cgs = prof["cgs"]
    dom = max(prof, key=lambda c: prof[c][1])
    print(f"# batched: {t_b / args.steps * 1e3:.1f} ms per batch, {rate_b:.0f} eigentriples/s, "
          f"mean d {info[:, 0].mean():.1f}, converged {info[:, 1].mean():.3f}", file=sys.stderr, flush=True)
    # one series at a time with the single-series path (plans built untimed)
    m = min(args.sample, ns)
    plans = [ssa.Plan(int(Ns[s]), Ls[s], k, device=dev, reorth=args.reorth) for s in range(m)]
    groups = [[i] for i in range(k)]

    def one(s):
        sg, U, V, inf = plans[s].truncated_svd(series[s], k)
        plans[s].reconstruct(sg, U, V, groups)
        return inf

    for s in range(min(4, m)):
        one(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infs = [one(s) for s in range(m)]
    torch.cuda.synchronize()
    t_1 = time.perf_counter() - t0
    d1 = [i.steps for i in infs]
    conv1 = sum(i.converged for i in infs)
    rate_1 = conv1 * k / t_1
    print(f"# one at a time: {m} series in {t_1:.3f} s, {rate_1:.0f} eigentriples/s, mean d {np.mean(d1):.1f}",
          file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_many(host, Ns, k, info, ns)
    out = {
        "metric": "eigentriples/s (many-series workload)",
        "value": rate_b,
        "unit": "eigentriples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_b / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{ns} series, N uniform in [2000, 20000], L = N/2, k = 16, two sinusoids + "
                               "trend + N(0, 0.1^2) (seeded); truncated SVD + 16 elementary reconstructions each",
                   "series": ns, "k": k, "reorth": "one-sided" if args.reorth else "full",
                   "parallelism": "single GPU"},
        "lanczos_steps_mean": float(info[:, 0].mean()),
        "converged_fraction": float(info[:, 1].mean()),
        "value_counts": "triples of series whose stopping rule held (equal accuracy); "
                        "value_all_series counts every series",
        "value_all_series": rate_b_all,
        "one_at_a_time": {"value": rate_1, "unit": "eigentriples/s", "series_timed": m,
                          "converged_fraction": conv1 / max(m, 1),
                          "lanczos_steps_mean": float(np.mean(d1)),
                          "path": "single-series plans (ssa_truncated_svd + ssa_reconstruct), one series after another"},
        "speedup_vs_one_at_a_time": rate_b / rate_1,
        "kernel_ms_per_batch": {c: v[1] / args.steps for c, v in prof.items()},
        "roofline": {
            "bound": "hbm",
            "kernel": "cgs (kb_cgs)" if dom == "cgs" else dom,
            "achieved": cgs_bytes / (ms_cgs / 1e3) / 1e9,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": cgs_bytes / (ms_cgs / 1e3) / 1e9 / HBM_PEAK_GBS,
            "traffic": traffic_per_launch("kb_cgs", "c3") if not args.reorth else None,
            "avg_launch_us": 1e3 * ms_cgs / max(n_cgs, 1),
            "alg_bytes_per_launch": cgs_bytes / max(n_cgs, 1),
            "note": "Gram-Schmidt launches (one per half-step, all series); bytes from each series' d",
        },
    }
    if cpu:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def cpu_baseline_many(host, Ns, k, info, ns):
    """Tier-B oracle (Lanczos with direct products, OpenMP) on a seeded sample of the series,
    each run for the GPU's own step count, extrapolated by N^2 d to the whole batch."""
    import numpy as np

    import oracle
    from paper_0911_4498_amd import inputs
    rng = np.random.default_rng(3)
    pick = [int(x) for x in sorted(rng.choice(ns, 24, replace=False))]
    t_s, w_s = 0.0, 0.0
    for s in pick:
        f, N, L = host[s]
        d = int(max(info[s, 0], k))
        t0 = time.perf_counter()
        oracle.lanczos_svd(f, L, k, inputs.start_vector(L, 4242), d_max=d, check_every=10**6)
        t_s += time.perf_counter() - t0
        w_s += float(N) * N * d
    d_all = np.maximum(info[:, 0].astype(np.float64), k)
    est = t_s / w_s * float(np.sum(Ns.astype(np.float64) ** 2 * d_all))
    return {
        "value": ns * k / est,
        "unit": "eigentriples/s",
        "cores": oracle.num_threads(),
        **host_cpu(),
        "kind": "oracle",
        "sample": (f"tier-B oracle (direct products) on {len(pick)} seeded series for their GPU step counts "
                   f"({t_s:.1f} s), extrapolated by N^2 d to all {ns} series; reconstructions not included"),
        "sample_seconds": round(t_s, 2),
    }


def served_stream(args, nreq, rates, quiet=False):
    """Served stream through ssa_server_*: requests with N <= args.batched_n_max go to the
    batched engine, longer ones to the server's long path (single-series plans bound to
    regions of the same pool, one check interval per tick).  Returns one result per rate."""
    import numpy as np
    import torch

    from paper_0911_4498_amd import inputs, ssa
    dev = torch.device("cuda:0")
    n_small_max = args.batched_n_max
    log = (lambda *a: None) if quiet else (lambda *a: print(*a, file=sys.stderr, flush=True))
    log(f"# generating {nreq} requests")
    reqs = []
    for r in range(nreq):
        f, N, L, k = inputs.c4_request(r)
        reqs.append((torch.tensor(f, device=dev), N, L, k))
    torch.cuda.synchronize()  # request series resident before any stream uses them
    srv = ssa.Server(n_max=n_small_max, k_max=32, slots=args.slots, pool_bytes=int(args.pool_gb * 2**30), device=dev,
                     reorth=args.reorth, n_long_max=1 << 20, long_slots=args.long_slots)

    def run_stream(rate, ids):
        arrivals = inputs.c4_arrivals(rate, len(ids))
        done_at = {}
        outs = {}
        t0 = time.perf_counter()
        nxt = 0
        while len(done_at) < len(ids):
            now = time.perf_counter() - t0
            while nxt < len(ids) and arrivals[nxt] <= now:
                r = ids[nxt]
                f, N, L, k = reqs[r]
                outs[r] = srv.submit(r, f, L, k, key=r)
                nxt += 1
            st = srv.status()
            if st["queued"] + st["active"] + st["finalizing"]:
                for r, _ in srv.step():
                    done_at[r] = time.perf_counter() - t0
                    outs.pop(r, None)
            else:
                time.sleep(min(1e-3, max(0.0, (arrivals[nxt] - now) if nxt < len(ids) else 1e-3)))
        lat = np.array([done_at[r] - arrivals[i] for i, r in enumerate(ids)])
        span = max(done_at.values()) - arrivals[0]
        is_small = np.array([reqs[r][1] <= n_small_max for r in ids])
        triples = sum(reqs[r][3] for r in ids)

        def pct(x, q):
            return float(np.percentile(x, q)) if len(x) else None

        return {"rate_req_s": rate, "requests": len(ids), "p50_s": pct(lat, 50), "p99_s": pct(lat, 99),
                "p50_short_s": pct(lat[is_small], 50), "p99_short_s": pct(lat[is_small], 99),
                "p50_long_s": pct(lat[~is_small], 50), "p99_long_s": pct(lat[~is_small], 99),
                "short_requests": int(is_small.sum()), "makespan_s": span,
                "eigentriples_per_s": triples / span}

    # warm-up: a few short and long requests, untimed
    log("# served warmup")
    small = [r for r in range(nreq) if reqs[r][1] <= n_small_max]
    run_stream(1000.0, small[:8] + [r for r in range(nreq) if r not in small][:2])
    results = []
    for rate in rates:
        log(f"# served rate {rate:.0f} req/s")
        res = run_stream(rate, list(range(nreq)))
        log(f"#   p50 {res['p50_s']:.3f} s  p99 {res['p99_s']:.3f} s  short p50 {res['p50_short_s']:.3f} s "
            f"p99 {res['p99_short_s']:.3f} s  long p50 {res['p50_long_s']:.3f} s  p99 {res['p99_long_s']:.3f} s  "
            f"{res['eigentriples_per_s']:.0f} eigentriples/s")
        results.append(res)
    srv.close()
    config = {"workload": f"Poisson stream of {nreq} requests per rate: N log-uniform in [1e3, 1e6], "
                          "L in {N/4, N/2}, k in [8, 32], c3 signals (seeded)",
              "short_path": f"continuous batching, N <= {n_small_max}, {args.slots} slots",
              "long_path": f"server long path: single-series plans bound to pool regions, {args.long_slots} slots, "
                           "one check interval per tick",
              "pool_gib": args.pool_gb, "reorth": "one-sided" if args.reorth else "full"}
    return results, config


def bench_served(args):
    """Served stream at each rate of --rates."""
    results, config = served_stream(args, args.requests, [float(x) for x in args.rates.split(",")])
    best = results[-1]
    out = {
        "metric": "p50/p99 served-SSA latency",
        "value": best["p99_s"],
        "unit": "s (p99, highest rate)",
        "n_gpus": 1,
        "steps": len(results),
        "warmup": 1,
        "ms_per_step": None,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {**config, "parallelism": "single GPU"},
        "rates": results,
    }
    print(json.dumps(out), flush=True)


def bench_hmatrix(args):
    """Structural-change detection: H-matrix time on the GPU (base-window SSAs on the batched
    path) against the CPU oracle, for the paper's comparison shape Q = N/2, B = T = N/4,
    L = B/2, I = {1, 2}."""
    import numpy as np
    import torch

    import oracle
    from paper_0911_4498_amd import inputs, ssa
    dev = torch.device("cuda:0")
    sizes = [int(x) for x in args.hm_sizes.split(",")]
    rows = []
    for N in sizes:
        B = T = N // 4
        L = B // 2
        f = inputs.hmatrix_series(N, N // 2, 5)
        fd = torch.tensor(f, device=dev)
        ssa.hmatrix(fd, B, T, L, [1, 2])  # warm-up
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            G = ssa.hmatrix(fd, B, T, L, [1, 2])
        torch.cuda.synchronize()
        t_gpu = (time.perf_counter() - t0) / reps
        row = {"N": N, "B": B, "T": T, "L": L, "windows": N - B + 1, "gpu_s": t_gpu}
        if N <= args.hm_oracle_max:
            t0 = time.perf_counter()
            ref = oracle.hmatrix(f, B, T, L, [1, 2])
            row["oracle_s"] = time.perf_counter() - t0
            row["oracle_cores"] = oracle.num_threads()
            row["max_abs_err_vs_oracle"] = float(np.abs(G.cpu().numpy() - ref).max())
        print(f"# N={N}: {row}", file=sys.stderr, flush=True)
        rows.append(row)
    out = {
        "metric": "H-matrix time (structural-change detection)",
        "value": rows[-1]["gpu_s"],
        "unit": "s",
        "n_gpus": 1,
        "higher_is_better": False,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "frequency change at Q = N/2 (period 10 -> 10.5) + 0.01 white noise; "
                               "B = T = N/4, L = B/2, I = {1, 2}"},
        "sizes": rows,
    }
    print(json.dumps(out), flush=True)


def bench_realizations(args):
    """Repeated realizations (the paper's bootstrap setting): rank-5 series, sigma = 5 white
    noise, L = N/2, rank-5 reconstructions of R realizations; GPU time against the CPU oracle."""
    import numpy as np
    import torch

    import oracle
    from paper_0911_4498_amd import inputs, ssa
    dev = torch.device("cuda:0")
    rows = []
    R = args.realizations
    for N in [int(x) for x in args.rs_sizes.split(",")]:
        L = N // 2
        f = inputs.rank5_example(N)
        F = f + 5.0 * np.stack([inputs.white(N, 100 + r) for r in range(R)])
        Fd = torch.tensor(F, device=dev)
        ssa.realizations(Fd, L, 5, truth=f)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mean, var, mse = ssa.realizations(Fd, L, 5, truth=f)
        torch.cuda.synchronize()
        row = {"N": N, "L": L, "R": R, "gpu_s": time.perf_counter() - t0,
               "mean_abs_bias": float(np.abs(mean.cpu().numpy() - f).mean()),
               "mean_var": float(var.mean().item()), "mean_mse": float(mse.mean().item())}
        if N <= args.rs_oracle_max:
            t0 = time.perf_counter()
            rm, rv, re = oracle.realization_stats(F, L, 5, f)
            row["oracle_s"] = time.perf_counter() - t0
            row["oracle_cores"] = oracle.num_threads()
            row["max_mean_diff_vs_oracle"] = float(np.abs(mean.cpu().numpy() - rm).max())
        print(f"# N={N}: {row}", file=sys.stderr, flush=True)
        rows.append(row)
    out = {
        "metric": "repeated-realization SSA time",
        "value": rows[-1]["gpu_s"],
        "unit": "s",
        "n_gpus": 1,
        "higher_is_better": False,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{R} realizations of the rank-5 series + N(0, 5^2) noise, L = N/2, "
                               "rank-5 reconstruction, per-point mean / variance / MSE"},
        "sizes": rows,
    }
    print(json.dumps(out), flush=True)


def bench_2d(args):
    """2D-SSA: seeded plane-wave arrays (three textures + trend + noise), window about half the
    array, k = 16 triples and 16 elementary reconstructions, at each of --s2-sizes; GPU time
    per solve, and the dense 2D oracle timed at the smallest size."""
    import numpy as np
    import torch

    import oracle
    from paper_0911_4498_amd import inputs, ssa
    dev = torch.device("cuda:0")
    k = 16
    rows = []
    sizes = [tuple(int(v) for v in x.split("x")) for x in args.s2_sizes.split(",")]
    for Nx, Ny in sizes:
        Lx, Ly = Nx // 2, Ny // 2
        F = inputs.array2d(Nx, Ny, seed=Nx + 7 * Ny)
        Fd = torch.tensor(F, device=dev)
        plan = ssa.Plan2D(Nx, Ny, Lx, Ly, k, device=dev)
        groups = [[i] for i in range(k)]

        def solve():
            s, U, V, info = plan.truncated_svd(Fd, k)
            plan.reconstruct(s, U, V, groups)
            return s, U, V, info

        for _ in range(max(1, args.warmup)):
            solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            s, U, V, info = solve()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        row = {"Nx": Nx, "Ny": Ny, "Lx": Lx, "Ly": Ly, "k": k, "gpu_s_per_solve": dt,
               "eigentriples_per_s": k / dt, "lanczos_steps": info.steps, "converged": info.converged,
               "trajectory_matrix": f"{Lx * Ly} x {(Nx - Lx + 1) * (Ny - Ly + 1)}"}
        if Lx * Ly <= args.s2_oracle_max:
            t0 = time.perf_counter()
            sA, UA, VA = oracle.ssa2d_dense(F, Lx, Ly, k)
            oracle.reconstruct_2d(Nx, Ny, Lx, Ly, sA, UA, VA, groups)
            row["oracle_s"] = time.perf_counter() - t0
            row["oracle_cores"] = oracle.num_threads()
            row["max_sigma_rel_diff_vs_oracle"] = float(np.max(np.abs(s.cpu().numpy() - sA) / sA))
        print(f"# {Nx}x{Ny}: {row}", file=sys.stderr, flush=True)
        rows.append(row)
        plan.close()
    out = {
        "metric": "eigentriples/s (2D-SSA)",
        "value": rows[-1]["eigentriples_per_s"],
        "unit": "eigentriples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D arrays of three plane waves + bilinear trend + N(0, 0.1^2), window "
                               "(Nx/2) x (Ny/2), k = 16 triples and 16 elementary reconstructions"},
        "sizes": rows,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pmc-copy", action="store_true", help="run the 256 MiB copy calibration first")
    ap.add_argument("--workload", choices=("single", "many", "served", "hmatrix", "realizations", "long", "2d"),
                    default="single")
    ap.add_argument("--s2-sizes", default="48x48,256x256,1024x1024", help="array sizes (2d workload)")
    ap.add_argument("--s2-oracle-max", type=int, default=600, help="largest Lx*Ly timed with the dense oracle")
    ap.add_argument("--check-every", type=int, default=0,
                    help="Lanczos steps between stopping tests (single workload; 0: the library default, 4)")
    ap.add_argument("--unfused", type=int, choices=(0, 1, 2), default=0,
                    help="1: six launches per Lanczos half-step; 2: the fused four (the reduction as "
                         "its own launch); 0: the fused path with each reduction folded into the next "
                         "pass 1 where it applies (A/B switch)")
    ap.add_argument("--reorth", type=int, choices=(0, 1), default=0,
                    help="0: full reorthogonalization, 1: one-sided (single, many and served workloads)")
    ap.add_argument("--schedule", choices=("table", "tune", "auto"), default="table",
                    help="FFT schedule of the single-series products: the stored tuner table, a tuner "
                         "run before the measurement, or the plan's automatic choice")
    ap.add_argument("--d-max", type=int, default=0, help="basis cap (long workload; default 125)")
    ap.add_argument("--restart-keep", type=int, default=0, help="Ritz pairs kept per restart (long; default 75)")
    ap.add_argument("--realizations", type=int, default=64, help="realizations per size (realizations workload)")
    ap.add_argument("--rs-sizes", default="1000,4000,16000", help="series lengths (realizations workload)")
    ap.add_argument("--rs-oracle-max", type=int, default=1000, help="largest N timed with the CPU oracle")
    ap.add_argument("--hm-sizes", default="400,1000,4000,8000", help="series lengths of the H-matrix workload")
    ap.add_argument("--hm-oracle-max", type=int, default=1000, help="largest N timed with the CPU oracle")
    ap.add_argument("--rates", default="100,1000", help="request rates of the served stream (req/s)")
    ap.add_argument("--requests", type=int, default=200, help="requests per rate (served stream)")
    ap.add_argument("--slots", type=int, default=256, help="server slots (served stream)")
    ap.add_argument("--pool-gb", type=float, default=24.0, help="server pool GiB (served stream)")
    ap.add_argument("--long-slots", type=int, default=4, help="server long-request slots (served stream)")
    ap.add_argument("--batched-n-max", type=int, default=8192,
                    help="longest series the server's batched engine takes (served stream; longer ones "
                         "take its single-series path; the engine allows up to 20480)")
    ap.add_argument("--served-requests", type=int, default=120,
                    help="requests of the bounded served leg of the default run (0: none)")
    ap.add_argument("--series", type=int, default=4096, help="series of the many-series workload")
    ap.add_argument("--sample", type=int, default=256, help="series timed one at a time (many-series workload)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the hot path runs on a single MI355X, and no "
              "multi-GPU path is built. Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    from paper_0911_4498_amd import ssa
    if not os.path.exists(ssa.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    if args.pmc_copy:
        copy_calibration()
    if args.workload in ("many", "served", "hmatrix", "realizations", "2d"):
        return {"many": bench_many, "served": bench_served, "hmatrix": bench_hmatrix,
                "realizations": bench_realizations, "2d": bench_2d}[args.workload](args)
    if args.workload == "long":
        return bench_long(args)
    from paper_0911_4498_amd import inputs
    f_np = inputs.c2_series(N)
    config = {"workload": "single long series: N=100000, L=50000, k=20, 5 sinusoids + exp trend + "
                          "AR(1) noise (seed 1002); truncated SVD + 20 elementary reconstructions",
              "N": N, "L": L, "k": K_TRIPLES, "reorth": "one-sided" if args.reorth else "full",
              "parallelism": "single GPU"}
    out = bench_plan(args, f_np, L, K_TRIPLES,
                     {"reorth": args.reorth, "unfused": args.unfused, "check_every": args.check_every},
                     "eigentriples/s (N=1e5, L=N/2, k=20)", config, traffic_per_launch)
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(f_np, int(round(out["lanczos_steps"])))
    if args.served_requests > 0:
        # a bounded served leg (the served-stream workload at one rate) beside the headline
        results, scfg = served_stream(args, args.served_requests, [100.0])
        out["served"] = {"metric": "p50/p99 served-SSA latency", **results[0], "config": scfg}
    print(json.dumps(out), flush=True)


def fft_schedule(args, Nw, Lw, f_dev):
    """Plan keywords of the products' FFT schedule and where they came from: the stored
    tuner table (default), a tuner run now (untimed), or the plan's automatic choice."""
    if args.schedule == "auto":
        return {}, "automatic"
    from paper_0911_4498_amd import autotune
    if args.schedule == "tune":
        e = autotune.tune(Nw, Lw, f_dev)
        print(f"# tuner: {e['candidates']} candidates in {e['tune_s']} s, best {e['us_per_pair']} us per "
              f"product pair, automatic {e['auto']['us_per_pair']}", file=sys.stderr, flush=True)
        return {key: e[key] for key in ("fft_mp", "fft_m1", "fft_cb")}, "tuned in this run (ssa_tune_fft)"
    sched = autotune.lookup(Nw, Lw)
    if sched is None:
        return {}, "automatic (no tuner table entry)"
    return sched, "tuner table (paper_0911_4498_amd/fft_schedules.json, ssa_tune_fft)"


def bench_plan(args, f_np, Lw, k, plan_kw, metric, config, traffic_fn):
    """One series through the single-series path: warm-up, one calibration solve with every
    kernel class event-timed (picks the dominant class), then the timed solves with the
    dominant class bracketed by HIP events on the plan's stream."""
    import numpy as np
    import torch

    from paper_0911_4498_amd import ssa
    dev = torch.device("cuda:0")
    Nw = len(f_np)
    f = torch.tensor(f_np, device=dev)
    sched, sched_src = fft_schedule(args, Nw, Lw, f)
    plan = ssa.Plan(Nw, Lw, k, device=dev, **plan_kw, **sched)
    d = plan.desc
    config = {**config, "fft": {"M_half": int(d.M) // 2, "M1": int(d.M1), "M2": int(d.M2), "CB": int(d.cb),
                                "schedule": sched_src}}
    print(f"# FFT schedule: M' = {d.M // 2} = {d.M1} x {d.M2}, CB = {d.cb} ({sched_src})", file=sys.stderr,
          flush=True)
    groups = [[i] for i in range(k)]
    steps_seen = []
    steps_run = []
    cycles = []
    launches = []

    def step():
        s, U, V, info = plan.truncated_svd(f, k)
        plan.reconstruct(s, U, V, groups)
        steps_seen.append(info.steps)
        steps_run.append(info.steps_run)
        cycles.append(info.thick_restarts)
        launches.append(info.half_step_launches)
        return info

    print(f"# warmup {args.warmup} steps", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    plan.profile_enable()
    step()
    calib = plan.profile_read()
    plan.profile_enable(on=False)
    candidates = ("pass1", "pass2", "pass3", "cgs_dots", "cgs_reduce", "cgs_update", "ritz",
                  "recon_pass1", "recon_pass2", "recon_pass3")
    dom = max(candidates, key=lambda c: calib[c][1])
    for name, (n, ms, b) in sorted(calib.items(), key=lambda kv: -kv[1][1]):
        if n:
            print(f"#   {name:12s} launches={n:6d} time={ms:9.3f} ms  avg={1e3 * ms / n:8.2f} us  "
                  f"alg={b / 1e6:9.3f} MB  {b / max(ms, 1e-9) / 1e6:8.1f} GB/s", file=sys.stderr)
    print(f"# dominant kernel class: {dom}", file=sys.stderr, flush=True)

    # one launch in eight of the dominant class bracketed by events: its mean duration is
    # measured live while the stream is disturbed as little as possible
    plan.profile_enable([dom], every=8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    starts = []
    for i in range(args.steps):
        starts.append(time.perf_counter())
        step()
        if Nw > 10**6:
            print(f"# timed step {i + 1}/{args.steps}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    t_timed = t_end - t0
    # per-step times: each solve ends with a host synchronization (its Ritz triples), so the
    # spacing of step starts is the step time; the last one ends at the final synchronization
    per_step = np.diff(np.array(starts + [t_end])) * 1e3
    prof = plan.profile_read()
    plan.profile_enable(on=False)
    print(f"# timed {args.steps} steps: {t_timed:.4f} s", file=sys.stderr, flush=True)
    # the embedding (spectrum of the series, once per series) on its own, outside the timed region
    for _ in range(3):
        plan.embed(f)
    torch.cuda.synchronize()
    te = time.perf_counter()
    for _ in range(10):
        plan.embed(f)
    torch.cuda.synchronize()
    embed_ms = (time.perf_counter() - te) / 10 * 1e3
    n_l, ms_l, b_l = prof[dom]
    achieved = (b_l / n_l) / (ms_l / n_l / 1e3) / 1e9 if n_l and ms_l > 0 else 0.0
    total_bytes = sum(v[2] for v in prof.values())
    return {
        "metric": metric,
        "value": k * args.steps / t_timed,
        "unit": "eigentriples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_timed / args.steps,
        "ms_per_step_median": float(np.median(per_step)),
        "ms_per_step_p90": float(np.percentile(per_step, 90)),
        "embed_ms": embed_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "dtype_detail": "FP32 FFTs, products and stored Lanczos vectors; FP64 Lanczos scalars, "
                        "Gram-Schmidt inner products and small bidiagonal SVD",
        "data": "synthetic",
        "config": config,
        "lanczos_steps": float(np.mean(steps_seen[-args.steps:])),
        "lanczos_steps_run": float(np.mean(steps_run[-args.steps:])),
        "thick_restarts": float(np.mean(cycles[-args.steps:])),
        "half_step_launches": sorted(set(launches[-args.steps:])),
        "matvecs_per_s": 2.0 * sum(steps_run[-args.steps:]) / t_timed,
        "hbm_gb_s_algorithmic": total_bytes / t_timed / 1e9,
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "kernel_name": (CLASS_KERNEL if plan_kw.get("unfused") == 1 else CLASS_KERNEL_FUSED).get(dom, dom),
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_fn(dom),
            "avg_launch_us": 1e3 * ms_l / max(n_l, 1),
            "alg_bytes_per_launch": b_l / max(n_l, 1),
        },
    }


def cpu_baseline_long(f, Lw, k, steps_gpu):
    """Oracle on a bounded sample of the N = 2^24 workload: direct row products of X and
    X^T and direct antidiagonal means at sampled positions, scaled to the GPU's steps
    (two products each) and to k Hankelizations of all N positions."""
    import numpy as np

    import oracle
    Nw = len(f)
    Kw = Nw - Lw + 1
    rng = np.random.default_rng(77)
    x = rng.normal(size=Kw)
    y = rng.normal(size=Lw)
    nrow = 8192  # about 10 s of direct products on 16 cores
    rows = np.sort(rng.choice(Lw, nrow, replace=False))
    cols = np.sort(rng.choice(Kw, nrow, replace=False))
    t0 = time.perf_counter()
    oracle.matvec_rows(f, Lw, x, rows)
    oracle.matvec_rows(f, Lw, y, cols, transpose=True)
    t_rows = time.perf_counter() - t0
    t_step = t_rows / (2 * nrow) * (Lw + Kw)
    pos = rng.choice(Nw, 2048, replace=False)
    t1 = time.perf_counter()
    oracle.hankelize_at(1.0, y, x, pos)
    t_pos = (time.perf_counter() - t1) / pos.size
    est = steps_gpu * t_step + k * Nw * t_pos
    return {
        "value": k / est,
        "unit": "eigentriples/s",
        "cores": oracle.num_threads(),
        **host_cpu(),
        "kind": "oracle",
        "sample": (f"direct products: {nrow} rows of X v and {nrow} of X^T u ({t_rows:.2f} s) scaled to "
                   f"{steps_gpu} steps of L + K rows; direct antidiagonal means at {pos.size} random positions "
                   f"({t_pos * 1e3:.2f} ms each) scaled to {k} x {Nw} positions"),
        "sample_seconds": round(t_rows + t_pos * pos.size, 2),
    }


def bench_long(args):
    """The very long series (N = 2^24, L = N/2, k = 50) with the basis capped by thick restart."""
    from paper_0911_4498_amd import inputs
    Nw = 2 ** 24
    Lw, k = Nw // 2, 50
    d_max = args.d_max or 125
    keep = args.restart_keep or 75
    print(f"# generating the N={Nw} series", file=sys.stderr, flush=True)
    f_np = inputs.c5_series(Nw)
    config = {"workload": f"very long series: N=2^24, L=N/2, k=50, 8 sinusoids + quadratic trend + "
                          f"N(0, 0.5^2) noise (seeded); thick restart with a {d_max}-column basis keeping "
                          f"{keep} Ritz pairs; truncated SVD + 50 elementary reconstructions",
              "N": Nw, "L": Lw, "k": k, "d_max": d_max, "restart_keep": keep, "parallelism": "single GPU"}
    out = bench_plan(args, f_np, Lw, k, {"d_max": d_max, "restart_keep": keep},
                     "eigentriples/s (N=2^24, L=N/2, k=50)", config, lambda cls: traffic_per_launch(cls, "c5"))
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_long(f_np, Lw, k, int(round(out["lanczos_steps_run"])))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
