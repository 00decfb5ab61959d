"""Benchmark of the sampled TR-ALS hot path on one MI355X.

A step is one sweep of Algorithm 2 (every core updated once: sample, sketch,
gather, normal equations, solve, new leverage table) over the default
workload, a 500 x 500 x 500 FP32 tensor built from random rank-(10,10,10)
TR cores plus 1% Gaussian noise, with J = 8192 samples per update (the
paper's synthetic-tensor experiment shape, Section 4.1.1).

Prints one JSON line: sampled rows/s (J * N rows per sweep), sweeps/s,
per-update latency percentiles, the dominant kernel's roofline (HIP events on
the library's stream) and the FP64 oracle's rate on a bounded sample of the
same workload on the host cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X dense FP32 matrix cores
PEAK_FP64_TFLOPS = 78.6
PEAK_BF16_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


CONTRACT_SOURCES = ("common.h", "normal_eq.hip")  # the contraction kernel's own sources


def kernel_source_sha():
    h = hashlib.sha256()
    for fn in CONTRACT_SOURCES:
        with open(os.path.join(ROOT, "paper_2010_08581_amd", "csrc", fn), "rb") as f:
            h.update(fn.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per launch of the dominant kernel from committed rocprofv3
    counter runs, if they were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "contract_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha") != kernel_source_sha() or rec.get("workload") != workload:
        return None
    return rec.get("bytes_per_launch")  # {"fetch", "write", "total"} in bytes


def cpu_baseline(X, init, cfg, budget_s):
    """FP64 oracle (test infrastructure) on a bounded number of updates."""
    from oracle import als as oals
    from oracle.leverage import core_table
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        blas_threads = None
    X64 = X.astype(np.float64)
    N = X.ndim
    J = cfg["samples"]
    cores = [np.array(c, dtype=np.float64) for c in init]
    tables = [None] + [core_table(cores[m]) for m in range(1, N)]
    t0 = time.perf_counter()
    done = 0
    while True:
        n = done % N
        cores[n], _, _ = oals.sampled_update(X64, cores, tables, n, J, cfg["seed"], 0, done)
        tables[n] = core_table(cores[n])
        done += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    cores_used = len(os.sched_getaffinity(0))
    return {
        "value": J * done / dt, "unit": "rows/s", "cores": blas_threads or cores_used, "kind": "oracle",
        "sample": f"{done} core updates (J={J}) of the same workload from the same initial cores, "
                  f"numpy FP64, {dt:.1f} s; host has {cores_used} usable cores",
    }


def method_forms(args, X, init, cfg):
    """Exact TR-ALS (Algorithm 1) and uniform sampling beside the leverage-score method, on the
    same tensor and initial cores, the same number of sweeps from fresh handles (the paper's
    protocol, Section 4.1: speedup at comparable error)."""
    import torch
    from paper_2010_08581_amd import TRALS
    dev = torch.device("cuda:0")
    ranks, J, prec = cfg["ranks"], cfg["samples"], cfg["precision"]
    S = args.method_sweeps
    out = {}
    Xt = torch.from_numpy(X).to(dev)
    for name, method, Jm in (("leverage", "leverage", J), ("uniform", "uniform", J),
                             ("uniform_4J", "uniform", 4 * J), ("exact", "exact", 0)):
        h = TRALS(Xt, ranks, Jm, seed=cfg["seed"], precision=prec, init_cores=init, method=method)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.sweep(S)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"method": method, "samples": Jm or None, "sweeps": S,
                     "ms_per_sweep": el / S * 1e3, "fit_error": h.fit_error()}
        log(f"{name}: {el / S * 1e3:.3f} ms/sweep, fit {out[name]['fit_error']:.5e}")
        del h
        torch.cuda.empty_cache()
    del Xt
    lev, ex = out["leverage"], out["exact"]
    out["speedup_leverage_vs_exact"] = ex["ms_per_sweep"] / lev["ms_per_sweep"]
    out["fit_ratio_leverage_vs_exact"] = lev["fit_error"] / ex["fit_error"]
    out["fit_ratio_uniform_vs_leverage"] = out["uniform"]["fit_error"] / lev["fit_error"]
    return out


def oscillatory_form():
    """Section 4.1.2 workload: 10-way 4^10 tensors of three oscillatory functions, ranks 10, the
    paper's protocol (exact TR-ALS until the error changes by less than 1e-3, at most 100
    sweeps; J from 2R^2 in steps of 100 until the sampled error is below 1.1x the exact one),
    both methods with the normalisation step (these runs are long enough for the unnormalised
    core scales to drift apart)."""
    import torch
    import synth
    from paper_2010_08581_amd import protocol
    out = {}
    R10 = (10,) * 10
    for name in synth.OSC_FUNCTIONS:
        X = synth.oscillatory_tensor(name)
        init = synth.random_cores(X.shape, R10, synth.rng_for(0, 3))
        Xt = torch.from_numpy(X).to("cuda:0")
        res = protocol.compare(Xt, R10, init, precision="f64", tol=1e-3, max_sweeps=100, factor=1.1,
                               J0=200, step=100, J_max=100000, normalize=True)
        out[name] = res
        log(f"oscillatory {name}: {res}")
        del Xt
        torch.cuda.empty_cache()
    return out


def serving_form(args):
    """Poisson stream of small decomposition requests (orders 3-5, sizes 32-256, ranks 3-12,
    J=2048, 5 sweeps, FP32, 1% noise) through the continuous-batching loop."""
    import synth
    from paper_2010_08581_amd.serve import TralsEngine, run, summarize
    eng = TralsEngine(synth.serving_true_cores, precision="f32", noise_rel=0.01, keep_cores=False)
    budget = 16 << 30
    eng.warmup(args.serve_slots)
    # each request carries its tensor's data (the true cores), made by the client beforehand
    reqs = [dict(r, true_cores=synth.serving_true_cores(r))
            for r in synth.serving_requests(args.serve_requests, rate=200.0, seed=0)]
    log(f"serving: {len(reqs)} requests at 200 req/s, {args.serve_slots} slots")
    res, wall, sched = run(eng, reqs, slots=args.serve_slots, mem_budget=budget)
    live = summarize(res, wall)
    live.update(rate_req_per_s=200.0, slots=args.serve_slots, peak_running=sched.peak_running)
    log(f"serving live: p50 {live['p50_ms']:.2f} ms p99 {live['p99_ms']:.2f} ms")
    # saturation: the same requests all at once, one at a time (plain) and concurrently
    burst = [dict(r, arrival=0.0) for r in reqs]
    res1, wall1, _ = run(eng, burst, slots=1, mem_budget=budget)
    resk, wallk, schedk = run(eng, burst, slots=args.serve_slots, mem_budget=budget)
    seq, conc = summarize(res1, wall1), summarize(resk, wallk)
    same = all(a.fit == b.fit for a, b in zip(res1, resk))
    log(f"serving saturated: sequential {seq['req_per_s']:.1f} req/s, concurrent {conc['req_per_s']:.1f} req/s")
    return {
        "workload": "Poisson 200 req/s; N in {3,4,5}, I_n in [32,256], R_n in [3,12], J=2048, 5 sweeps, "
                    "fp32, 1% noise, generated source",
        "live": live,
        "saturated_sequential": seq,
        "saturated_concurrent": dict(conc, slots=args.serve_slots, peak_running=schedk.peak_running),
        "speedup_concurrent_vs_sequential": conc["req_per_s"] / seq["req_per_s"],
        "fit_identical_alone_and_mixed": same,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--latency-updates", type=int, default=60)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16-form", action="store_true")
    ap.add_argument("--no-serving-form", action="store_true")
    ap.add_argument("--no-method-forms", action="store_true")
    ap.add_argument("--method-sweeps", type=int, default=10)
    ap.add_argument("--no-oscillatory-form", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-slots", type=int, default=8)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the method runs on one GPU)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2010_08581_amd import TRALS

    cfg = dict(synth.CONFIGS[args.config])
    dims, ranks, J, prec = cfg["dims"], cfg["ranks"], cfg["samples"], cfg["precision"]
    N = len(dims)
    log(f"generating {cfg['name']} {dims} ranks {ranks}")
    t = time.perf_counter()
    X, _, init = synth.make_config(args.config, dtype=np.float64 if prec == "f64" else np.float32)
    log(f"generated in {time.perf_counter() - t:.1f} s")
    dev = torch.device("cuda:0")
    Xt = torch.from_numpy(X).to(dev)
    h = TRALS(Xt, ranks, J, seed=cfg["seed"], precision=prec, init_cores=init)
    del Xt
    torch.cuda.synchronize()
    log("handle created")
    if args.warmup:
        h.sweep(args.warmup)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} sweeps done")

    # timed region: K sweeps, no events between the kernels (an event record on the stream
    # costs a gap of ~10 us between back-to-back kernels)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.sweep(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    log(f"timed {args.steps} sweeps in {elapsed:.3f} s")
    # per-kernel durations: the same K sweeps again with HIP events around every kernel group,
    # recorded on the library's stream
    h.profile(True)
    h.sweep(args.steps)
    kern = {}
    for k in ("draw", "contract", "reduce", "factor", "solve", "table"):
        ms, cnt = h.profile_read(k)
        kern[k] = {"ms_per_launch": ms / max(cnt, 1), "launches": cnt}
    h.profile(False)

    # per-update latency (one core update = sample + sketch + normal equations + solve + table)
    lat = []
    for _ in range(args.latency_updates):
        a = time.perf_counter()
        h.step(1)
        lat.append(time.perf_counter() - a)
    lat_us = np.array(lat) * 1e6
    fit = h.fit_error()
    log(f"latency done, fit {fit:.4e}")

    rows = J * N * args.steps
    value = rows / elapsed
    esz = {"f64": 8, "f32": 4, "bf16": 2}[prec]
    P = [ranks[(n - 1) % N] * ranks[n] for n in range(N)]
    # the method's contraction: fused fiber gather + [A^T A | A^T X~] (algorithmic FLOPs: B plus
    # the lower triangle of H); FP32 data are multiplied on the FP64 matrix cores (exact widening)
    avg_s = kern["contract"]["ms_per_launch"] * 1e-3
    flops = np.mean([2.0 * J * P[n] * dims[n] + J * P[n] * (P[n] + 1.0) for n in range(N)])
    gbytes = np.mean([J * dims[n] * esz for n in range(N)])
    peak = {"f64": PEAK_FP64_TFLOPS, "f32": PEAK_FP64_TFLOPS, "bf16": PEAK_BF16_TFLOPS}[prec]
    achieved = flops / avg_s / 1e12
    traffic = measured_traffic(cfg["name"])
    roofline = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": traffic["total"] if traffic else None,
                "traffic_fetch_write": [traffic["fetch"], traffic["write"]] if traffic else None,
                "algorithmic_bytes": gbytes,
                "kernel": "k_normal_eq (fiber gather + [A^T A | A^T X~] on matrix cores)",
                "gather_GBps": gbytes / avg_s / 1e9,
                "gather_hbm_frac": gbytes / avg_s / 1e9 / PEAK_HBM_GBS}
    bytes_sweep = J * sum(dims) * esz
    out = {
        "metric": "sampled ALS rows/s", "value": value, "unit": "rows/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": prec,
        "data": "synthetic",
        "config": {"workload": cfg["name"], "dims": list(dims), "ranks": list(ranks), "samples": J,
                   "noise": f"{cfg['noise'][0]} {cfg['noise'][1]}", "seed": cfg["seed"],
                   "step": "one sweep (N core updates)"},
        "sweeps_per_s": args.steps / elapsed,
        "hbm_frac": bytes_sweep / (elapsed / args.steps) / (PEAK_HBM_GBS * 1e9),
        "update_latency_us": {"p50": float(np.percentile(lat_us, 50)), "p99": float(np.percentile(lat_us, 99))},
        "fit_error": fit,
        "kernels_ms_per_launch": {k: v["ms_per_launch"] for k, v in kern.items()},
        "roofline": roofline,
    }
    if prec == "f32" and not args.no_bf16_form:
        # the BF16 form on the same input, initial cores and number of sweeps
        del h
        torch.cuda.empty_cache()
        Xt = torch.from_numpy(X).to(dev)
        hb = TRALS(Xt, ranks, J, seed=cfg["seed"], precision="bf16", init_cores=init)
        del Xt
        if args.warmup:
            hb.sweep(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hb.sweep(args.steps)
        torch.cuda.synchronize()
        eb = time.perf_counter() - t0
        hb.profile(True)
        hb.sweep(args.steps)
        ms, cnt = hb.profile_read("contract")
        hb.profile(False)
        hb.step(args.latency_updates)
        fb = hb.fit_error()
        out["forms"] = {"bf16": {
            "value": J * N * args.steps / eb, "unit": "rows/s", "ms_per_step": eb / args.steps * 1e3,
            "speedup_vs_f32": elapsed / eb, "fit_error": fb, "fit_rel_diff_vs_f32": abs(fb - fit) / fit,
            "contract_ms_per_launch": ms / max(cnt, 1),
            "contract_gather_GBps": np.mean([J * dims[n] * 2 for n in range(N)]) / (ms / max(cnt, 1) * 1e-3) / 1e9,
        }}
        log(f"bf16 form: {eb / args.steps * 1e3:.3f} ms/sweep, fit {fb:.4e}")
    if not args.no_method_forms and J * 4 <= (1 << 24):
        h = hb = None  # noqa: F841
        torch.cuda.empty_cache()
        out.setdefault("forms", {})["methods"] = method_forms(args, X, init, cfg)
    if not args.no_oscillatory_form:
        h = hb = None  # noqa: F841
        torch.cuda.empty_cache()
        out.setdefault("forms", {})["oscillatory"] = oscillatory_form()
    if not args.no_serving_form:
        h = hb = None  # noqa: F841 (releases the handles' workspaces)
        torch.cuda.empty_cache()
        out.setdefault("forms", {})["serving"] = serving_form(args)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(X, init, cfg, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
