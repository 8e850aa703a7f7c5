"""Benchmark of the EBC greedy hot path on one MI355X.

One step = one whole pass of the hot path over the resident ground set:
dataset residency/precompute (norms, L({e0}), padded copy) followed by
greedy to cardinality k with all n points as candidates at every step
(marginal gains on the MFMA units -> window -> float64 re-score -> m_v
update -> f(S_t)). Default workload: n = 100000 points from a 20-component
Gaussian mixture in d = 100, k = 50, float32 distances.

metric  candidate x point distance evaluations per second over the whole
        greedy run, counting sum_{t<k} n*(n-t) pairs per step (already
        selected points are not counted).

Prints one JSON line; see the design notes for the roofline and the
cpu_baseline definitions.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published dense matrix peaks (TFLOP/s) per distance dtype
PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0, "f16": 2500.0, "fp8": 5000.0}
WORKLOADS = {
    # name: (generator kwargs, description)
    "gmm20_n100000_d100_k50": ("greedy_fp32", {"seed": 2}),
    "gmm50+out_n200000_d64_k100": ("precision_sweep", {"seed": 3}),
    "normal_n1000_d16_k5": ("small_normal", {"seed": 0}),
    "batched512_bf16_k20": ("batched_instances", {"seed": 4}),
    "serving_curves_d64_bf16": ("serving_requests", {"seed": 5}),
    "paper_sets_n50000_l5000_k10_d100": ("paper_sets", {"seed": 6}),
    "paper_sets_sweep_d100": ("paper_sets", {"seed": 6}),
    "curves_n1000_d3524_k50": ("case_study_curves", {"seed": 8}),
    "sieves_curves_n1000_d3524_k50": ("case_study_curves", {"seed": 8}),
    "sievestream_curves_n1000_d3524_k50": ("case_study_curves", {"seed": 8}),
}


def pairs_per_greedy(n: int, k: int) -> int:
    return sum(n * (n - t) for t in range(k))


def cpu_baseline(x, n: int, target_s: float = 12.0) -> dict:
    """The FP64 oracle's gains loop (plain C, OpenMP over candidates) timed on
    a bounded sample: the first step's gains for a prefix of the candidates."""
    import numpy as np

    from oracle import build_ref, ref
    if not os.path.exists(build_ref.LIB):
        build_ref.build()
    m = ref.min_dist(x, [])
    nc = 256
    while True:
        cand = np.arange(nc, dtype=np.int32)
        t0 = time.perf_counter()
        ref.gains(x, m, cand)
        dt = time.perf_counter() - t0
        if dt >= target_s or nc >= n:
            break
        nc = min(n, max(nc * 2, int(nc * target_s / max(dt, 1e-3))))
    return {"value": nc * n / dt, "unit": "pair-evals/s", "cores": ref.threads(), "kind": "oracle",
            "sample": f"float64 gains of the first {nc} candidates against all {n} points at S={{}} "
                      f"(one greedy step's work for {nc} candidates; {dt:.1f} s)"}


def paper_style_cpu(x, n: int, value: float) -> dict:
    """The paper's comparison (Table 1): single- and multi-threaded CPU runs in
    single precision; here the gains loop (oracle/ebc_ref.c, ebc_ref_gains_f32)
    on a bounded prefix of the candidates (about 2 s each), with the speedup
    of `value` (pair-evals/s) over each."""
    import numpy as np

    from oracle import ref
    m = ref.min_dist(x, [])
    out = {}
    for label, threads in (("st", 1), ("mt", ref.threads())):
        nc = 16
        while True:
            cand = np.arange(nc, dtype=np.int32)
            t0 = time.perf_counter()
            ref.gains_f32(x, m, cand, threads)
            el = time.perf_counter() - t0
            if el >= 2.0 or nc >= n:
                break
            nc = min(n, max(nc * 2, int(nc * 3.0 / max(el, 1e-3))))
        rate = nc * n / el
        out[label] = {"pair_evals_per_s": rate, "threads": threads, "candidates": nc, "speedup": value / rate}
    return out


def counters_traffic(kernel: str, workload: str, dtype: str, variant: int):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 --pmc
    summary (FETCH_SIZE, WRITE_SIZE scaled by a plain-copy calibration), or
    None if none was taken on this workload, dtype and variant, or the
    kernel's source has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "counters.json")
    try:
        recs = json.load(open(path))["records"]
    except (OSError, KeyError, ValueError):
        return None
    for rec in recs:
        if (rec.get("kernel"), rec.get("workload"), rec.get("dtype"), rec.get("variant")) != \
                (kernel, workload, dtype, variant):
            continue
        try:
            src = open(os.path.join(ROOT, rec["source"]), "rb").read()
        except OSError:
            return None
        if hashlib.sha256(src).hexdigest()[:16] != rec["source_sha256_16"]:
            return None
        return int(rec["hbm_bytes_per_launch"])
    return None


def bench_batched(args):
    """512 independent instances (n ~ U{2000..50000}, d in {8..128}, k = 20,
    BF16 distances) advanced together by ebc_greedy_batched in graph mode;
    tile variants autotuned per (dtype, row padding, size bucket)."""
    import numpy as np
    import torch

    from paper_2105_12026_amd import ebc, workloads

    dev = torch.device("cuda:0")
    t_gen = time.perf_counter()
    insts = workloads.batched_instances(seed=4, count=512)
    dss = []
    for p in insts:
        dss.append(ebc.Dataset(torch.from_numpy(p.x).to(dev), dtype=args.dtype if args.dtype != "f32" else "bf16"))
    print(f"# generated and uploaded {len(dss)} instances in {time.perf_counter() - t_gen:.1f} s",
          file=sys.stderr, flush=True)
    tuned = {}
    for ds in dss:
        r = ds.autotune(reps=2)
        tuned[(ds.dtype, ds.info()["k_pad"])] = r["variant"]
    torch.cuda.synchronize()
    batch = ebc.Batch(dss)
    batch.set_graph(True)
    ks = [p.k for p in insts]
    outs = None
    for _ in range(args.warmup):
        outs = batch.greedy(ks)
    torch.cuda.synchronize()
    with ClockSampler() as clk:
        t0 = time.perf_counter()
        for _ in range(args.steps):
            outs = batch.greedy(ks, outs=[(o[0], o[1], o[2]) for o in outs] if outs else None)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    for ds in dss:
        ds.sync()
    pairs = sum(pairs_per_greedy(p.n, p.k) for p in insts)
    flops = sum(2.0 * p.d * pairs_per_greedy(p.n, p.k) for p in insts)
    ms = elapsed * 1e3 / args.steps
    achieved = flops / (ms * 1e-3) / 1e12
    dt = dss[0].dtype
    info = batch.info()
    out = {
        "metric": "candidate x point distance evals/s (batched greedy, all candidates)",
        "value": pairs * args.steps / elapsed, "unit": "pair-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dt, "data": "synthetic",
        "config": {"workload": "batched512_bf16_k20", "instances": len(insts), "k": 20,
                   "n_range": [min(p.n for p in insts), max(p.n for p in insts)],
                   "d_set": sorted({p.d for p in insts}), "step": "reset + 20 ticks, one graph",
                   "tuned_variants": {f"{k[0]}/k_pad{k[1]}": v for k, v in sorted(tuned.items())},
                   "buckets": info["buckets"], "gains_workgroups_per_tick": info["gains_workgroups_per_tick"]},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[dt], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_TFLOPS[dt], 4), "traffic": None,
                     "kernel": "whole batched step (all kernels), algorithmic 2*d flops per pair"},
    }
    ghz = clk.mean()
    if ghz:
        out["roofline"]["clock_ghz_sampled"] = round(ghz, 3)
        out["roofline"]["frac_at_sampled_clock"] = round(achieved / (PEAK_TFLOPS[dt] * ghz / 2.4), 4)
    print(json.dumps(out), flush=True)


def bench_serving(args):
    """Serving: summarisation requests of process curves (n ~ U{5000..100000},
    d = 64, k ~ U{5..50}, BF16 distances) through the serving core. The
    closed-loop capacity mu (all requests queued at once) is measured first;
    then Poisson streams at 0.3, 0.7 and 1.1 mu, each reporting p50/p99
    latency from arrival to the result on the host and completed req/s.
    The stream cycles through a pool of distinct seeded requests."""
    import numpy as np
    import torch

    from paper_2105_12026_amd import ebc, serving, workloads

    pool_n = args.serving_pool
    t_gen = time.perf_counter()
    pool = workloads.serving_requests(seed=5, count=pool_n)
    print(f"# generated {pool_n} requests in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    dt = args.dtype if args.dtype != "f32" else "bf16"
    # autotune the gains variant per (dtype, row length, size bucket) seen in the pool
    for p in pool[:8]:
        ds = ebc.Dataset(torch.from_numpy(p.x).cuda(), dtype=dt)
        ds.autotune(reps=2)
        ds.close()
    torch.cuda.synchronize()
    arena_bytes = args.serving_arena_gib << 30
    sv = ebc.Server(arena_bytes, max_slots=args.serving_slots)
    payloads = [(p.x, p.k) for p in pool]
    flops_of = lambda ps: sum(2.0 * 64 * pairs_per_greedy(x.shape[0], k) for x, k in ps)
    # warm-up, then closed loop
    serving.run_closed_loop(sv, payloads[:4], dtype=dt)
    closed = payloads * max(1, args.steps)
    recs, c0, c1 = serving.run_closed_loop(sv, closed, dtype=dt)
    closed_s = c1 - c0
    mu = len(closed) / closed_s
    closed_sum = serving.summarize(recs, c0)
    achieved = flops_of(closed) / closed_s / 1e12
    print(f"# closed loop: {len(closed)} requests in {closed_s:.2f} s, mu = {mu:.1f} req/s", file=sys.stderr,
          flush=True)
    rates = {}
    for j, frac in enumerate((0.3, 0.7, 1.1)):
        count = args.serving_requests
        stream = [payloads[i % pool_n] for i in range(count)]
        arr = workloads.poisson_arrivals(5 + j, frac * mu, count)
        recs, t0 = serving.run_open_loop(
            sv, stream, arr, dtype=dt,
            progress=lambda done, total: print(f"# rate {frac} mu: {done}/{total} finished", file=sys.stderr,
                                               flush=True))
        summ = serving.summarize(recs, t0)
        summ["offered_req_per_s"] = frac * mu
        rates[f"{frac}mu"] = {k: (round(v, 5) if isinstance(v, float) else v) for k, v in summ.items()}
        print(f"# rate {frac} mu: {summ}", file=sys.stderr, flush=True)
    st = sv.stats()
    sv.close()
    out = {
        "metric": "requests/s (serving, closed-loop capacity), p50/p99 latency at 0.3/0.7/1.1 of it",
        "value": mu, "unit": "req/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": closed_s * 1e3 / max(1, args.steps), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dt, "data": "synthetic",
        "config": {"workload": "serving_curves_d64_bf16", "pool": pool_n, "closed_loop_requests": len(closed),
                   "requests_per_rate": args.serving_requests, "max_slots": args.serving_slots,
                   "arena_gib": args.serving_arena_gib, "ticks": st["ticks"],
                   "closed_loop_latency": {k: (round(v, 5) if isinstance(v, float) else v)
                                           for k, v in closed_sum.items()},
                   "rates": rates},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[dt], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_TFLOPS[dt], 4), "traffic": None,
                     "kernel": "whole serving loop in the closed-loop run, algorithmic 2*d flops per pair"},
    }
    print(json.dumps(out), flush=True)


def bench_sets(args):
    """Multi-set evaluation (ebc_eval_sets) in the shape of the paper's runtime
    sweep: |V| = 50000 N(0,1) points in d = 100, l = 5000 random sets of 10.
    One step = one ebc_eval_sets call over all l sets (inputs resident).
    Metric: (set member, point) pairs per second, l * k_set * |V| per call."""
    import numpy as np
    import torch

    from paper_2105_12026_amd import ebc, workloads

    kw = {}
    for part in (args.sets_shape or "").split(","):
        if part:
            key, val = part.split("=")
            kw[key] = int(val)
    p = workloads.paper_sets(seed=6, **kw)
    n, d = p.n, p.d
    l = len(p.offsets) - 1
    nnz = int(p.offsets[-1])
    dev = torch.device("cuda:0")
    dt = args.dtype
    ds = ebc.Dataset(torch.from_numpy(p.x).to(dev), dtype=dt)
    off = torch.from_numpy(p.offsets).to(dev)
    idx = torch.from_numpy(p.idx).to(dev)
    out = torch.empty(l, dtype=torch.float64, device=dev)
    lowp = dt != "f32"  # dot products in the dataset's dtype (the paper's FP16 variant)
    for _ in range(args.warmup):
        ds.eval_sets(off, idx, out=out, in_dtype=lowp)
    torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ds.eval_sets(off, idx, out=out, in_dtype=lowp)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ds.sync()
    ms = float(np.median(times))
    pairs = float(nnz) * n
    achieved = 2.0 * d * pairs / (ms * 1e-3) / 1e12
    res = {
        "metric": "set-member x point distance evals/s (ebc_eval_sets, all sets)",
        "value": pairs / (ms * 1e-3), "unit": "pair-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dt, "data": "synthetic",
        "config": {"workload": p.name, "n": n, "d": d, "sets": l, "set_size": nnz // max(l, 1),
                   "ms_min": float(np.min(times)), "ms_max": float(np.max(times)),
                   "step": "one ebc_eval_sets call over all sets"},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[dt], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_TFLOPS[dt], 4), "traffic": None,
                     "kernel": "whole ebc_eval_sets call, algorithmic 2*d flops per (member, point) pair"},
    }
    if not args.no_cpu_baseline:
        from oracle import build_ref, ref
        if not os.path.exists(build_ref.LIB):
            build_ref.build()
        ns = 8
        while True:
            t0 = time.perf_counter()
            ref.eval_sets(p.x, p.offsets[:ns + 1], p.idx[:int(p.offsets[ns])])
            dt = time.perf_counter() - t0
            if dt >= 8.0 or ns >= l:
                break
            ns = min(l, max(ns * 2, int(ns * 10.0 / max(dt, 1e-3))))
        res["cpu_baseline"] = {"value": float(p.offsets[ns]) * n / dt, "unit": "pair-evals/s",
                               "cores": ref.threads(), "kind": "oracle",
                               "sample": f"float64 f of the first {ns} sets ({dt:.1f} s)"}
        # The paper's own comparison (Table 1): single- and multi-threaded CPU
        # runs of Alg. 1 in single precision; speedups of this GPU line over both.
        paper_cpu = {}
        for label, threads in (("st", 1), ("mt", ref.threads())):
            ns = 4
            while True:
                t0 = time.perf_counter()
                ref.eval_sets_f32(p.x, p.offsets[:ns + 1], p.idx[:int(p.offsets[ns])], threads)
                el = time.perf_counter() - t0
                if el >= 2.0 or ns >= l:
                    break
                ns = min(l, max(ns * 2, int(ns * 3.0 / max(el, 1e-3))))
            rate = float(p.offsets[ns]) * n / el
            paper_cpu[label] = {"pair_evals_per_s": rate, "threads": threads, "sets": ns,
                                "speedup": res["value"] / rate}
        res["paper_style_cpu"] = paper_cpu
    print(json.dumps(res), flush=True)


def bench_sieves(args):
    """Three Sieves (ebc_three_sieves; workload sievestream_*: Sieve Streaming,
    ebc_sieve_streaming, one summary per guess) over the case-study shape: 1000 process
    curves of length 3524 streamed in index order into a summary of k = 50
    (grid ratio eps = 0.1, T = 5 rejections per threshold step; the paper's
    case study, Sec. 6, runs Three Sieves on N = 1000, d = 3524 series). One
    step = one call from S = {} (inputs resident). Metric: (examined point,
    ground point) pairs per second, i.e. points examined * n per call."""
    import numpy as np
    import torch

    from paper_2105_12026_amd import ebc, workloads

    p = workloads.case_study_curves(seed=8)
    n, d, k = p.n, p.d, p.k
    stream_all = args.workload.startswith("sievestream")  # Sieve Streaming: one summary per guess
    eps, T = (0.1, 5) if not stream_all else (0.1, 0)
    dev = torch.device("cuda:0")
    ds = ebc.Dataset(torch.from_numpy(p.x).to(dev), dtype=args.dtype)

    def run():
        if stream_all:
            sel, f, _, seen = ds.sieve_streaming(k, eps)
            return sel, f, seen
        return ds.three_sieves(k, eps, T)

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    times, seen, acc = [], 0, 0
    for _ in range(args.steps):
        t0 = time.perf_counter()
        sel, f, seen = run()
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
        acc = int(sel.numel())
    ds.sync()
    ms = float(np.median(times))
    pairs = float(seen) * n
    # each (examined point, ground point) distance: d float64 subtractions
    # and d fused multiply-adds (3d flops) on the vector ALUs
    achieved = 3.0 * d * pairs / (ms * 1e-3) / 1e12
    res = {
        "metric": "examined-point x point distance evals/s ("
                  + ("sieve streaming, best summary" if stream_all else "three sieves, one summary") + ")",
        "value": pairs / (ms * 1e-3), "unit": "pair-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "d": d, "k": k, "eps": eps, "T": T,
                   "dataset_dtype": args.dtype,
                   "accepted": acc, "examined": seen, "f_last": float(f[-1]) if acc else 0.0,
                   "ms_min": float(np.min(times)), "ms_max": float(np.max(times)),
                   "step": ("one ebc_sieve_streaming call" if stream_all else "one ebc_three_sieves call")
                   + ", stream in index order"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": 78.6,
                     "unit": "TFLOP/s", "frac": round(achieved / 78.6, 4), "traffic": None,
                     "kernel": "whole call: float64 distances of each examined point (3*d flops per pair, "
                               "FP64 vector peak) and the on-device decision walk"},
    }
    if not args.no_cpu_baseline:
        # the float64 oracle (NumPy, as it stands) on a bounded prefix of the stream
        from oracle import build_ref, ebc_oracle, ref
        if not os.path.exists(build_ref.LIB):
            build_ref.build()
        mx = float(np.max(ref.gains(p.x, ref.min_dist(p.x, []))))  # largest singleton value (C oracle)
        limit = 8 if stream_all else 120
        t0 = time.perf_counter()
        if stream_all:
            _, _, _, o_seen = ebc_oracle.sieve_streaming(p.x, k, eps, m=mx, order=range(limit))
        else:
            _, _, _, o_seen = ebc_oracle.three_sieves(p.x, k, eps, T, m=mx, order=range(limit))
        el = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": o_seen * n / el, "unit": "pair-evals/s", "cores": 1, "kind": "oracle",
                               "sample": f"float64 NumPy oracle on the first {limit} points of the stream "
                                         f"({o_seen} examined, {el:.1f} s; the largest singleton value given)"}
    print(json.dumps(res), flush=True)


def bench_sets_sweep(args):
    """The paper's runtime sweep (Sec. 5.1) on ebc_eval_sets: from the defaults
    |V| = 50000, l = 5000, k = 10 (d = 100, N(0,1) data, random sets), vary
    one of N, l, k at a time over the paper's ranges. Each point: median of
    args.steps calls after args.warmup. One JSON line with every point."""
    import numpy as np
    import torch

    from paper_2105_12026_amd import ebc, workloads

    series = {
        "N": [("n", v) for v in range(1000, 400001, 28500)],
        "l": [("l", v) for v in range(1000, 26071, 2785)],
        "k": [("set_size", v) for v in range(10, 431, 35)],
    }
    dev = torch.device("cuda:0")
    points = []
    for name, pts in series.items():
        for key, val in pts:
            kw = {"n": 50000, "l": 5000, "set_size": 10}
            kw[key] = val
            p = workloads.paper_sets(seed=6, **kw)
            ds = ebc.Dataset(torch.from_numpy(p.x).to(dev), dtype="f32")
            off = torch.from_numpy(p.offsets).to(dev)
            idx = torch.from_numpy(p.idx).to(dev)
            out = torch.empty(kw["l"], dtype=torch.float64, device=dev)
            for _ in range(args.warmup):
                ds.eval_sets(off, idx, out=out)
            times = []
            for _ in range(args.steps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                ds.eval_sets(off, idx, out=out)
                e1.record()
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            ds.sync()
            ms = float(np.median(times))
            pairs = float(kw["n"]) * kw["l"] * kw["set_size"]
            tf = 2.0 * 100 * pairs / (ms * 1e-3) / 1e12
            points.append({"vary": name, **kw, "ms": round(ms, 4), "pair_evals_per_s": pairs / (ms * 1e-3),
                           "tflops": round(tf, 2)})
            print(f"# {name}={val}: {ms:.3f} ms, {tf:.1f} TFLOP/s", file=sys.stderr, flush=True)
            del ds, off, idx, out
    best = max(pt["pair_evals_per_s"] for pt in points)
    dflt = [pt for pt in points if pt["n"] == 50000 and pt["l"] == 5000 and pt["set_size"] == 10][0]
    res = {
        "metric": "set-member x point distance evals/s (ebc_eval_sets, paper sweep)",
        "value": dflt["pair_evals_per_s"], "unit": "pair-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dflt["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "paper_sets_sweep_d100", "points": points, "best_pair_evals_per_s": best},
        "roofline": {"bound": "mfma", "achieved": dflt["tflops"], "peak": PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
                     "frac": round(dflt["tflops"] / PEAK_TFLOPS["f32"], 4), "traffic": None,
                     "kernel": "whole ebc_eval_sets call at the defaults, 2*d flops per (member, point) pair"},
    }
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="gmm20_n100000_d100_k50", choices=sorted(WORKLOADS))
    ap.add_argument("--dtype", default="f32", choices=sorted(PEAK_TFLOPS))
    ap.add_argument("--variant", type=int, default=None, help="tile variant of the gains kernel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="bf16,f16,fp8",
                    help="reduced-precision legs of an FP32 greedy line (comma-separated dtypes, '' for none)")
    ap.add_argument("--leg-steps", type=int, default=5, help="timed runs per reduced-precision leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--sets-shape", default="", help="paper_sets overrides, e.g. n=50000,l=5000,set_size=10")
    ap.add_argument("--serving-pool", type=int, default=24, help="distinct requests the serving stream cycles")
    ap.add_argument("--serving-requests", type=int, default=150, help="requests per arrival rate")
    ap.add_argument("--serving-slots", type=int, default=64)
    ap.add_argument("--serving-arena-gib", type=int, default=32)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is a design note only",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    if args.workload.startswith("batched"):
        bench_batched(args)
        return
    if args.workload.startswith("serving"):
        bench_serving(args)
        return
    if args.workload.startswith("sieves"):
        bench_sieves(args)
        return
    if args.workload == "paper_sets_sweep_d100":
        bench_sets_sweep(args)
        return
    if args.workload.startswith("paper_sets"):
        bench_sets(args)
        return

    import numpy as np
    import torch

    from paper_2105_12026_amd import ebc, workloads

    gen, kw = WORKLOADS[args.workload]
    p = getattr(workloads, gen)(**kw)
    n, d, k = p.n, p.d, p.k
    dev = torch.device("cuda:0")
    x = torch.from_numpy(p.x).to(dev)
    stream = torch.cuda.current_stream()
    print(f"# workload {args.workload}: n={n} d={d} k={k}", file=sys.stderr, flush=True)
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print("# copy calibration: 268435456 bytes read, 268435456 bytes written", file=sys.stderr, flush=True)

    golden = load_golden(args.workload, p)
    run = timed_greedy(ebc, torch, x, n, d, k, args.dtype, args.variant, args.steps, args.warmup, stream)
    ms_per_step = run["ms"]
    pairs = pairs_per_greedy(n, k)
    value = pairs / (ms_per_step * 1e-3)
    roofline = run["roofline"]
    roofline["traffic"] = counters_traffic(roofline["kernel"], args.workload, args.dtype, run["variant"])

    out = {
        "metric": "candidate x point distance evals/s (greedy, all candidates)",
        "value": value, "unit": "pair-evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "d": d, "k": k, "distance_dtype": args.dtype,
                   "variant": run["variant"],
                   "candidates": "all n points every step", "step": "residency + greedy k"},
        "greedy_ms": ms_per_step, "gains_kernel_ms_total_per_step": run["gains_ms_per_run"],
        "rest_of_step_ms_per_step": run["select_ms_per_run"],
        "window_max": run["window_max"], "f_last": float(run["f"][-1]), "sel_head": run["sel"][:5],
        "roofline": roofline,
    }
    if golden is not None:
        out["parity"] = parity_vs_golden(np, run, golden, args.dtype)
    if args.legs and args.dtype == "f32":
        # the metric compares FP32 with reduced-precision distances: the same
        # greedy run per dtype (timed like the main line, fewer runs), with
        # its speed-up over FP32 and its f error and selection agreement
        # against the stored float64 oracle run
        legs = {}
        for dt in [v for v in args.legs.split(",") if v]:
            r = timed_greedy(ebc, torch, x, n, d, k, dt, None, args.leg_steps, 1, stream)
            leg = {"ms_per_run": round(r["ms"], 3), "pair_evals_per_s": pairs / (r["ms"] * 1e-3),
                   "speedup_vs_f32": round(ms_per_step / r["ms"], 3), "variant": r["variant"],
                   "window_max": r["window_max"],
                   "roofline": {k2: r["roofline"][k2] for k2 in ("kernel", "achieved", "peak", "frac",
                                                                   "avg_launch_ms", "clock_ghz_sampled",
                                                                   "frac_at_sampled_clock")
                                if k2 in r["roofline"]}}
            if golden is not None:
                leg["parity"] = parity_vs_golden(np, r, golden, dt)
            legs[dt] = leg
            print(f"# leg {dt}: {leg}", file=sys.stderr, flush=True)
        out["legs"] = legs
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p.x, n)
        out["paper_style_cpu"] = paper_style_cpu(p.x, n, value)
    print(json.dumps(out), flush=True)


GOLDEN = {"gmm20_n100000_d100_k50": "gmm20_n100000_d100_k50.json",
          "gmm50+out_n200000_d64_k100": "gmm50+out_n200000_d64_k100.json",
          "normal_n1000_d16_k5": "normal_n1000_d16.json"}


def load_golden(workload, p):
    """The stored float64 oracle run of this workload (tests/golden/, written
    by tests/golden/make_golden.py from the oracle), if its input matches."""
    from paper_2105_12026_amd import workloads
    name = GOLDEN.get(workload)
    if not name:
        return None
    try:
        g = json.load(open(os.path.join(ROOT, "tests", "golden", name)))
    except OSError:
        return None
    return g if g.get("sha256_x") == workloads.sha256_of(p.x) and "sel" in g else None


def parity_vs_golden(np, run, golden, dt):
    """Selections and f(S_t) of a timed run against the stored oracle run:
    FP32 must select the oracle's points in the oracle's order; every dtype
    reports the largest relative f error over the common prefix (where the
    sets are equal, so f must agree to float64 rounding), the agreement, the
    common prefix and the final quality gap."""
    sel, f = run["sel"], np.asarray(run["f"])
    rsel, rf = golden["sel"], np.asarray(golden["f"])
    k = len(rsel)
    prefix = next((i for i in range(k) if sel[i] != rsel[i]), k)
    f_err = float(np.max(np.abs(f[:prefix] - rf[:prefix]) / np.abs(rf[:prefix]))) if prefix else None
    return {"sel_equal": sel == rsel, "agreement": len(set(sel) & set(rsel)) / k, "common_prefix": prefix,
            "max_rel_f_err_on_prefix": f_err, "quality_gap": float((rf[-1] - f[-1]) / rf[-1]),
            "reference": "tests/golden (float64 oracle run)"}


class ClockSampler:
    """Samples the GPU's graphics clock (amdsmi, mean over the XCDs) every
    `period` seconds from a side thread while the timed region runs; mean()
    is the average in GHz, or None when no sample could be read. Used to
    state each roofline fraction also against the peak at the measured clock
    (the published peaks assume 2.4 GHz)."""

    def __init__(self, period: float = 0.01):
        import threading
        self.period, self.samples, self._stop = period, [], threading.Event()
        self._thread = None
        try:
            import amdsmi
            amdsmi.amdsmi_init()
            self._smi = amdsmi
            self._h = amdsmi.amdsmi_get_processor_handles()[0]
        except Exception:
            self._smi = None

    def _read(self):
        m = self._smi.amdsmi_get_gpu_metrics_info(self._h)
        vals = m.get("current_gfxclks")
        if not isinstance(vals, (list, tuple)):
            vals = [m.get("current_gfxclk")]
        vals = [float(v) for v in vals if isinstance(v, (int, float)) and 0 < v < 10000]
        return sum(vals) / len(vals) / 1e3 if vals else None

    def _run(self):
        while not self._stop.is_set():
            try:
                v = self._read()
                if v:
                    self.samples.append(v)
            except Exception:
                return
            self._stop.wait(self.period)

    def __enter__(self):
        import threading
        if self._smi is not None:
            self._thread = threading.Thread(target=self._run, daemon=True)
            self._thread.start()
        return self

    def __exit__(self, *exc):
        self._stop.set()
        if self._thread is not None:
            self._thread.join(timeout=2.0)
        if self._smi is not None:
            try:
                self._smi.amdsmi_shut_down()
            except Exception:
                pass

    def mean(self):
        return sum(self.samples) / len(self.samples) if self.samples else None


def timed_greedy(ebc, torch, x, n, d, k, dtype, variant, steps, warmup, stream):
    """`warmup` untimed then `steps` timed runs of one step (dataset residency
    + greedy k) in `dtype`, with the per-launch gains-kernel time from the
    library's HIP events on the launch stream."""
    dev = x.device
    sel = torch.empty(k, dtype=torch.int32, device=dev)
    f = torch.empty(k, dtype=torch.float64, device=dev)
    gain = torch.empty(k, dtype=torch.float64, device=dev)
    # gains tile variant: as given, else the autotuner's choice for this
    # (dtype, row length, size), timed once before the measured steps
    variant_used = 0
    if variant is not None:
        variant_used = variant
    elif dtype != "f32" and d <= 128:  # long rows have a single kernel shape
        tds = ebc.Dataset(x, dtype=dtype, stream=stream)
        variant_used = tds.autotune(reps=3, stream=stream)["variant"]
        tds.sync(stream)
        tds.close()

    def one_step(profile: bool):
        ds = ebc.Dataset(x, dtype=dtype, stream=stream)
        if dtype != "f32":
            ds.set_variant(variant_used)
        if profile:
            ds.profile(True)
        ds.greedy(k, stream=stream, sel=sel, f=f, gain=gain)
        return ds

    keep = []
    for _ in range(warmup):
        keep.append(one_step(False))
    torch.cuda.synchronize()
    for ds in keep:
        ds.sync()
    keep.clear()
    torch.cuda.synchronize()
    with ClockSampler() as clk:
        t0 = time.perf_counter()
        for _ in range(steps):
            keep.append(one_step(True))
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    prof = {"gains_ms": 0.0, "select_ms": 0.0, "gains_launches": 0, "steps": 0}
    window_max = 0
    for ds in keep:
        st = ds.sync()
        window_max = max(window_max, st["window_max"])
        pr = ds.profile_read()
        for key in prof:
            prof[key] += pr[key]
    # roofline of the dominant kernel (marginal gains on the MFMA units):
    # algorithmic flops per launch = 2*d per (candidate, point) pair, with
    # the already-selected candidates not counted, averaged over the steps;
    # padding of d and the affine chunk are not counted.
    gains_avg_ms = prof["gains_ms"] / max(prof["gains_launches"], 1)
    flops_per_launch = 2.0 * d * pairs_per_greedy(n, k) / k
    achieved = flops_per_launch / (gains_avg_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[dtype]
    if d > 128:
        kname = "k_gains_wide"
    else:
        kname = "k_gains_f32" if dtype == "f32" else \
            {3: "k_gains_lp_pp", 4: "k_gains_lp_sp"}.get(variant_used, "k_gains_lp")
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                "kernel": kname, "avg_launch_ms": round(gains_avg_ms, 4),
                "flops_per_launch": flops_per_launch}
    ghz = clk.mean()
    if ghz:
        # the same fraction against the peak scaled to the clock sampled during the timed runs
        roofline["clock_ghz_sampled"] = round(ghz, 3)
        roofline["frac_at_sampled_clock"] = round(achieved / (peak * ghz / 2.4), 4)
    return {"ms": elapsed * 1e3 / steps, "variant": variant_used, "window_max": window_max,
            "gains_ms_per_run": prof["gains_ms"] / steps, "select_ms_per_run": prof["select_ms"] / steps,
            "sel": sel.cpu().numpy().tolist(), "f": f.cpu().numpy().tolist(), "roofline": roofline}


if __name__ == "__main__":
    main()
