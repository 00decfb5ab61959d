"""Benchmark of the sampled TR-ALS hot path on one MI355X.

A step is one sweep of Algorithm 2 (every core updated once: sample, sketch, gather, normal
equations, solve, new leverage table).  The default workload is the largest one: a
video-shaped 240 x 320 x 3 x 2000 FP32 tensor (smooth Gaussian blobs on linear trajectories
plus uniform noise, the stand-in for the paper's colour-video data, Section 4.1.3), TR ranks 20,
J = 16384 samples per core update.

Prints one JSON line: sampled rows/s (J * N rows per sweep), sweeps/s, per-sweep and
per-update latency percentiles, the dominant kernel's roofline (HIP events on the library's
stream), the per-update error of the FP32 path and of the BF16 form against the FP64 oracle
(lockstep on a bounded number of updates), the other forms (500^3 workload, methods, the
paper's protocol on the oscillatory functions, serving) and the FP64 oracle's rate on a
bounded sample of the headline workload on the host cores.
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X dense FP32 matrix cores
PEAK_FP64_TFLOPS = 78.6
PEAK_BF16_TFLOPS = 2500.0
X3_PRODUCTS = 8  # BF16 slice products per FP32 product in the three-slice contraction
PEAK_HBM_GBS = 8000.0
METRIC = "sampled ALS rows/s & sweeps/s (HBM GB/s frac); p50/p99 solve latency"


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


def measured_traffic(workload, precision):
    """HBM bytes per launch of the contraction from committed rocprofv3 counter runs, if they
    were taken on the current kernel sources for this workload and precision."""
    path = os.path.join(ROOT, "profiles", "contract_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        recs = json.load(f)
    for rec in recs.get("records", []):
        if (rec.get("workload") == workload and rec.get("precision") == precision
                and rec.get("source_sha") == kernel_source_sha()):
            return rec.get("bytes_per_launch")  # {"fetch", "write", "total"} in bytes
    return None


def host_info():
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        return max([d.get("num_threads", 1) for d in info] or [1]), sorted({d.get("internal_api", "?") for d in info})
    except Exception:
        return None, []


def cpu_baseline(X, init, cfg, budget_s):
    """FP64 oracle (test infrastructure) on a bounded number of updates of the same workload
    from the same initial cores, timed on the host."""
    from oracle import als as oals
    from oracle.leverage import core_table
    X64 = X.astype(np.float64)
    threads, apis = blas_threads()
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
        if done >= 2 and time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    model, ncores = host_info()
    return {
        "value": J * done / dt, "unit": "rows/s", "cores": threads or ncores, "kind": "oracle",
        "sample": f"{done} core updates (J={J}, modes 0..{min(done, N) - 1} in order) of the {cfg['name']} "
                  f"workload from the same initial cores, numpy FP64 oracle, {dt:.1f} s",
        "cpu_model": model, "host_cores": ncores, "blas_threads": threads, "blas": apis,
    }


def slice_err(got, want):
    """(worst over lateral slices of max|g - o| / max|o|, Frobenius ratio) of one core."""
    d = np.abs(got - want).max(axis=(0, 2))
    s = np.abs(want).max(axis=(0, 2))
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(s > 0, d / np.where(s > 0, s, 1.0), np.where(d > 0, np.inf, 0.0))
    return float(r.max()), float(np.linalg.norm(got - want) / np.linalg.norm(want))


def oracle_lockstep(h, X64, cfg, updates):
    """Per-update error of the handle's path against the FP64 oracle: before each update the
    oracle takes the handle's cores, draws and solves; indices compared bit for bit, weights and
    the new core (per lateral slice) relative to the oracle's."""
    from oracle import als as oals
    N = X64.ndim
    J = cfg["samples"]
    recs = []
    for _ in range(updates):
        u = h.update_counter
        n = u % N
        before = [c.cpu().numpy() for c in h.get_cores()]
        h.step(1)
        idx_g, w_g = h.last_samples()
        core_o, idx_o, w_o = oals.lockstep_update(X64, before, n, J, cfg["seed"], 0, u)
        worst, fro = slice_err(h.get_cores()[n].cpu().numpy(), core_o)
        recs.append({"update": u, "mode": n, "indices_equal": bool(np.array_equal(idx_g, idx_o)),
                     "weights_max_rel": float(np.max(np.abs(w_g - w_o) / w_o)),
                     "core_worst_slice_rel": worst, "core_fro_rel": fro})
    return {"updates": recs,
            "indices_bit_exact": all(r["indices_equal"] for r in recs),
            "max_core_worst_slice_rel": max(r["core_worst_slice_rel"] for r in recs),
            "max_core_fro_rel": max(r["core_fro_rel"] for r in recs)}


def time_sweeps(h, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.sweep(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def kernel_groups(h, steps):
    h.profile(True)
    h.sweep(steps)
    kern = {}
    for k in ("draw", "contract", "reduce", "factor", "solve", "table"):
        ms, cnt = h.profile_read(k)
        kern[k] = {"ms_per_launch": ms / max(cnt, 1), "launches": cnt, "ms_per_sweep": ms / steps}
    h.profile(False)
    return kern


def latencies(h, sweeps, updates):
    """Per-sweep and per-update wall latencies (each call synchronises), in microseconds."""
    lat_s = []
    for _ in range(sweeps):
        a = time.perf_counter()
        h.sweep(1)
        lat_s.append(time.perf_counter() - a)
    lat_u = []
    for _ in range(updates):
        a = time.perf_counter()
        h.step(1)
        lat_u.append(time.perf_counter() - a)
    pct = lambda v: {"p50": float(np.percentile(v, 50)), "p99": float(np.percentile(v, 99)),  # noqa: E731
                     "samples": len(v)}
    return pct(np.array(lat_s) * 1e6), pct(np.array(lat_u) * 1e6)


def contraction_work(cfg):
    """Algorithmic FLOPs and gathered bytes of one contraction launch, averaged over the N
    updates of a sweep: 2 J P I_n (B = A^T X~) + J P (P + 1) (lower triangle of H = A^T A),
    and J I_n s (the sampled fibers)."""
    dims, ranks, J = cfg["dims"], cfg["ranks"], cfg["samples"]
    N = len(dims)
    P = [ranks[(n - 1) % N] * ranks[n] for n in range(N)]
    flops = float(np.mean([2.0 * J * P[n] * dims[n] + J * P[n] * (P[n] + 1.0) for n in range(N)]))
    return flops, [J * dims[n] for n in range(N)]


def run_workload(args, cfg, X, init, prec, steps, warmup, lat_sweeps, lat_updates):
    """Timed sweeps, kernel groups and latencies of one precision on one workload."""
    import torch
    from paper_2010_08581_amd import TRALS
    Xt = torch.from_numpy(X).to("cuda:0")
    h = TRALS(Xt, cfg["ranks"], cfg["samples"], seed=cfg["seed"], precision=prec, init_cores=init)
    del Xt
    torch.cuda.synchronize()
    if warmup:
        h.sweep(warmup)
    # timed region: the sweeps alone, no events between the kernels (an event record on the
    # stream costs a gap of ~10 us between back-to-back kernels)
    elapsed = time_sweeps(h, steps)
    kern = kernel_groups(h, steps)
    lat_s, lat_u = latencies(h, lat_sweeps, lat_updates)
    fit = h.fit_error()
    N = len(cfg["dims"])
    res = {"precision": prec, "steps": steps, "elapsed_s": elapsed, "ms_per_sweep": elapsed / steps * 1e3,
           "rows_per_s": cfg["samples"] * N * steps / elapsed, "sweeps_per_s": steps / elapsed,
           "fit_error": fit, "kernels": kern, "sweep_latency_us": lat_s, "update_latency_us": lat_u}
    return h, res


def method_forms(args, X, init, cfg):
    """Exact TR-ALS (Algorithm 1) and uniform sampling beside the leverage-score method, on the
    same tensor and initial cores, the same number of sweeps from fresh handles."""
    import torch
    from paper_2010_08581_amd import TRALS
    dev = torch.device("cuda:0")
    ranks, J, prec = cfg["ranks"], cfg["samples"], cfg["precision"]
    S = args.method_sweeps
    out = {"workload": cfg["name"]}
    Xt = torch.from_numpy(X).to(dev)
    for name, method, Jm in (("leverage", "leverage", J), ("uniform", "uniform", J),
                             ("uniform_4J", "uniform", 4 * J), ("exact", "exact", 0)):
        h = TRALS(Xt, ranks, Jm, seed=cfg["seed"], precision=prec, init_cores=init, method=method)
        el = time_sweeps(h, S)
        out[name] = {"method": method, "samples": Jm or None, "sweeps": S,
                     "ms_per_sweep": el / S * 1e3, "fit_error": h.fit_error()}
        log(f"{name}: {el / S * 1e3:.3f} ms/sweep, fit {out[name]['fit_error']:.5e}")
        h.close()
        del h
        torch.cuda.empty_cache()
    del Xt
    lev, ex = out["leverage"], out["exact"]
    out["speedup_leverage_vs_exact"] = ex["ms_per_sweep"] / lev["ms_per_sweep"]
    out["fit_ratio_leverage_vs_exact"] = lev["fit_error"] / ex["fit_error"]
    out["fit_ratio_uniform_vs_leverage"] = out["uniform"]["fit_error"] / lev["fit_error"]
    return out


def oscillatory_form(args):
    """Section 4.1.2 workload: 10-way 4^10 tensors of three oscillatory functions, ranks 10, the
    paper's protocol: exact TR-ALS until the relative error changes by less than 1e-3 (at most
    100 sweeps) gives S; both methods then run 2 S sweeps from the same cores; J walks up from
    2 R^2 = 200 in steps of 100 to the first J whose error is below 1.1 x the exact error (J_max
    bounds the walk).  Both methods with the normalisation step (these runs are long enough for
    the unnormalised core scales to drift apart)."""
    import torch
    import synth
    from paper_2010_08581_amd import protocol
    out = {}
    R10 = (10,) * 10
    for name in synth.OSC_FUNCTIONS:
        X = synth.oscillatory_tensor(name)
        init = synth.random_cores(X.shape, R10, synth.rng_for(0, 3))
        Xt = torch.from_numpy(X).to("cuda:0")
        t0 = time.perf_counter()
        res = protocol.compare(Xt, R10, init, precision="f64", tol=1e-3, max_sweeps=100, factor=1.1,
                               J0=200, step=100, J_max=args.osc_j_max, normalize=True, search="walk")
        res["wall_s"] = time.perf_counter() - t0
        out[name] = res
        log(f"oscillatory {name}: {res['outcome']} ({res['runs']} runs, {res['wall_s']:.1f} s)")
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
    order = {r["id"]: len(r["dims"]) for r in reqs}

    def by_order(results):
        out = {}
        for N in sorted(set(order.values())):
            f = np.array([x.fit for x in results if x.error is None and x.fit is not None and order[x.id] == N])
            if f.size:
                out[str(N)] = {"requests": int(f.size), "fit_p10": float(np.percentile(f, 10)),
                               "fit_median": float(np.median(f)), "fit_p90": float(np.percentile(f, 90))}
        return out
    # The same requests with a sample count that lets them converge.  Theorem 3 asks for J above
    # prod_j R_j^2 times a log factor, exponential in the order; the method converges well below
    # that, and on these random-core tensors 20 sweeps from N(0,1) cores reach the noise floor
    # once J is a few times prod_j R_j (at J = 2048 order-4 and order-5 requests stay at a fit
    # of about 1, order-3 ones converge).  J is capped to bound memory and time; requests whose
    # rule exceeds the cap are counted apart.
    def enough(r):
        want = 4 * int(np.prod(r["ranks"]))
        J = min(args.serve_j_cap, max(2048, -(-want // 1024) * 1024))
        return dict(r, samples=J, sweeps=args.serve_converged_sweeps, capped=want > args.serve_j_cap)
    conv = [enough(r) for r in burst]
    resc, wallc, schedc = run(eng, conv, slots=args.serve_slots, mem_budget=budget)
    convs = summarize(resc, wallc)
    by_id = {r["id"]: r for r in conv}
    conv_by_order = by_order(resc)
    for N, d in conv_by_order.items():
        mine = [x for x in resc if x.error is None and x.fit is not None and order[x.id] == int(N)]
        d["converged_frac"] = float(np.mean([x.fit < 1e-2 for x in mine]))
        d["J_median"] = int(np.median([by_id[x.id]["samples"] for x in mine]))
        d["capped"] = int(sum(by_id[x.id]["capped"] for x in mine))
        d["converged_frac_uncapped"] = float(np.mean([x.fit < 1e-2 for x in mine if not by_id[x.id]["capped"]]
                                                     or [np.nan]))
    log(f"serving J = 4 prod R, {args.serve_converged_sweeps} sweeps: {convs['req_per_s']:.1f} req/s, "
        + ", ".join(f"order {N} converged {d['converged_frac']:.2f}" for N, d in conv_by_order.items()))
    return {
        "workload": "Poisson 200 req/s; N in {3,4,5}, I_n in [32,256], R_n in [3,12], J=2048, 5 sweeps, "
                    "fp32, 1% noise, generated source; fit = ||TR(G) - TR(G*)|| / ||TR(G*)||",
        "live": live,
        "saturated_sequential": seq,
        "saturated_concurrent": dict(conc, slots=args.serve_slots, peak_running=schedk.peak_running),
        "speedup_concurrent_vs_sequential": conc["req_per_s"] / seq["req_per_s"],
        "fit_identical_alone_and_mixed": same,
        "fit_by_order_5_sweeps": by_order(resk),
        "sufficient_samples": dict(convs, rule="J = clamp(4 prod_j R_j, 2048, cap), rounded up to 1024",
                                   J_cap=args.serve_j_cap, sweeps=args.serve_converged_sweeps,
                                   slots=args.serve_slots, fit_by_order=conv_by_order),
    }


def workload_form(args, key):
    """A second workload (FP32 and the BF16 form, same input and initial cores): rows/s and fit."""
    import torch
    import synth
    cfg = dict(synth.CONFIGS[key])
    prec = cfg["precision"]
    X, _, init = synth.make_config(key, dtype=np.float64 if prec == "f64" else np.float32)
    out = {"workload": cfg["name"], "dims": list(cfg["dims"]), "ranks": list(cfg["ranks"]), "samples": cfg["samples"]}
    h, res = run_workload(args, cfg, X, init, prec, args.steps, args.warmup, 50, 30)
    h.close()
    out[prec] = res
    log(f"{cfg['name']} {prec}: {res['ms_per_sweep']:.3f} ms/sweep, fit {res['fit_error']:.5e}")
    if prec == "f32":
        torch.cuda.empty_cache()
        hb, rb = run_workload(args, cfg, X, init, "bf16", args.steps, args.warmup, 50, 30)
        hb.close()
        rb["speedup_vs_f32"] = res["ms_per_sweep"] / rb["ms_per_sweep"]
        rb["fit_rel_diff_vs_f32"] = abs(rb["fit_error"] - res["fit_error"]) / res["fit_error"]
        out["bf16"] = rb
        log(f"{cfg['name']} bf16: {rb['ms_per_sweep']:.3f} ms/sweep, fit {rb['fit_error']:.5e}")
    torch.cuda.empty_cache()
    return out, X, init, cfg


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c4")
    ap.add_argument("--latency-sweeps", type=int, default=200)
    ap.add_argument("--latency-updates", type=int, default=60)
    ap.add_argument("--oracle-updates", type=int, default=4,
                    help="lockstep updates against the FP64 oracle per precision (0: none)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16-form", action="store_true")
    ap.add_argument("--forms", default="c2", help="comma-separated extra workloads (\"\" for none)")
    ap.add_argument("--no-serving-form", action="store_true")
    ap.add_argument("--no-method-forms", action="store_true")
    ap.add_argument("--method-sweeps", type=int, default=10)
    ap.add_argument("--no-oscillatory-form", action="store_true")
    ap.add_argument("--osc-j-max", type=int, default=3000)
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-converged-sweeps", type=int, default=20)
    ap.add_argument("--serve-j-cap", type=int, default=262144)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the method runs on one GPU)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth

    cfg = dict(synth.CONFIGS[args.config])
    dims, ranks, J, prec = cfg["dims"], cfg["ranks"], cfg["samples"], cfg["precision"]
    N = len(dims)
    log(f"generating {cfg['name']} {dims} ranks {ranks}")
    t = time.perf_counter()
    X, _, init = synth.make_config(args.config, dtype=np.float64 if prec == "f64" else np.float32)
    log(f"generated in {time.perf_counter() - t:.1f} s")
    h, res = run_workload(args, cfg, X, init, prec, args.steps, args.warmup, args.latency_sweeps,
                          args.latency_updates)
    log(f"{cfg['name']} {prec}: {res['ms_per_sweep']:.3f} ms/sweep ({args.steps} sweeps), fit {res['fit_error']:.4e}")
    esz = {"f64": 8, "f32": 4, "bf16": 2}[prec]
    flops, rows_in = contraction_work(cfg)
    kern = res["kernels"]
    avg_s = kern["contract"]["ms_per_launch"] * 1e-3
    gbytes = float(np.mean(rows_in)) * esz
    # FP32 path: up to P = 128 FP32 data widen exactly onto the FP64 matrix cores (priced
    # against the FP64 matrix peak); above, three 8-bit slices of each FP32 operand meet on the
    # BF16 matrix cores (eight of the nine slice products per FP32 product, the ninth below
    # 2^-34 of the block maxima), priced against the dense FP32 matrix peak, the precision the
    # products have
    Pmax = max(ranks[(n - 1) % N] * ranks[n] for n in range(N))
    three_slice = prec == "f32" and Pmax > 128
    peak = {"f64": PEAK_FP64_TFLOPS, "f32": PEAK_FP32_TFLOPS if three_slice else PEAK_FP64_TFLOPS,
            "bf16": PEAK_BF16_TFLOPS}[prec]
    achieved = flops / avg_s / 1e12
    traffic = measured_traffic(cfg["name"], prec)
    roofline = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": traffic["total"] if traffic else None,
                "traffic_fetch_write": [traffic["fetch"], traffic["write"]] if traffic else None,
                "algorithmic_flops": flops, "algorithmic_bytes": gbytes,
                "kernel": ("k_x3_split + k_normal_eq_x3 (the sketch rows and the gathered, weighted fibers "
                           "split into three 8-bit slices once per update, then [A^T A | A^T X~] from the slices "
                           "on BF16 matrix cores, eight slice products, FP64 block sums; timed from the first "
                           "kernel's start to the second's end)") if three_slice else
                          "k_normal_eq (fiber gather + [A^T A | A^T X~] on FP64 matrix cores)",
                "kernel_share_of_sweep": kern["contract"]["ms_per_sweep"] / res["ms_per_sweep"],
                "gather_GBps": gbytes / avg_s / 1e9,
                "gather_hbm_frac": gbytes / avg_s / 1e9 / PEAK_HBM_GBS}
    if three_slice:
        roofline["executed_bf16_tflops"] = X3_PRODUCTS * achieved
        roofline["executed_bf16_frac"] = X3_PRODUCTS * achieved / PEAK_BF16_TFLOPS
    bytes_sweep = J * sum(dims) * esz
    out = {
        "metric": METRIC, "value": res["rows_per_s"], "unit": "rows/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["ms_per_sweep"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": prec,
        "data": "synthetic",
        "config": {"workload": cfg["name"], "dims": list(dims), "ranks": list(ranks), "samples": J,
                   "noise": f"{cfg['noise'][0]} {cfg['noise'][1]}", "seed": cfg["seed"],
                   "step": "one sweep (N core updates)"},
        "sweeps_per_s": res["sweeps_per_s"],
        "hbm_frac": bytes_sweep / (res["ms_per_sweep"] * 1e-3) / (PEAK_HBM_GBS * 1e9),
        "sweep_latency_us": res["sweep_latency_us"],
        "update_latency_us": res["update_latency_us"],
        "fit_error": res["fit_error"],
        "kernels_ms_per_sweep": {k: v["ms_per_sweep"] for k, v in kern.items()},
        "kernels_ms_per_launch": {k: v["ms_per_launch"] for k, v in kern.items()},
        "roofline": roofline,
        "forms": {},
    }
    X64 = X.astype(np.float64) if args.oracle_updates > 0 else None
    if args.oracle_updates > 0:
        log("lockstep against the FP64 oracle ...")
        out["error_vs_oracle"] = {prec: oracle_lockstep(h, X64, cfg, args.oracle_updates)}
    h.close()
    del h
    torch.cuda.empty_cache()
    if prec == "f32" and not args.no_bf16_form:
        # the BF16 form on the same input, initial cores and number of sweeps
        hb, rb = run_workload(args, cfg, X, init, "bf16", args.steps, args.warmup, 50, 30)
        rb["speedup_vs_f32"] = res["ms_per_sweep"] / rb["ms_per_sweep"]
        rb["fit_rel_diff_vs_f32"] = abs(rb["fit_error"] - res["fit_error"]) / res["fit_error"]
        rb["contract_gather_GBps"] = float(np.mean(rows_in)) * 2 / (rb["kernels"]["contract"]["ms_per_launch"] * 1e-3) / 1e9
        if args.oracle_updates > 0:
            out["error_vs_oracle"]["bf16"] = oracle_lockstep(hb, X64, cfg, args.oracle_updates)
        hb.close()
        del hb
        out["forms"]["bf16"] = rb
        log(f"bf16 form: {rb['ms_per_sweep']:.3f} ms/sweep ({rb['speedup_vs_f32']:.2f}x), fit {rb['fit_error']:.4e}")
        torch.cuda.empty_cache()
        # the BF16 form with its subchain products on BF16 matrix cores as well
        hc, rc = run_workload(args, cfg, X, init, "bf16c", args.steps, args.warmup, 10, 10)
        rc["speedup_vs_f32"] = res["ms_per_sweep"] / rc["ms_per_sweep"]
        rc["fit_rel_diff_vs_f32"] = abs(rc["fit_error"] - res["fit_error"]) / res["fit_error"]
        if args.oracle_updates > 0:
            out["error_vs_oracle"]["bf16c"] = oracle_lockstep(hc, X64, cfg, args.oracle_updates)
        hc.close()
        del hc
        out["forms"]["bf16_chains"] = rc
        log(f"bf16 form, chains on matrix cores: {rc['ms_per_sweep']:.3f} ms/sweep ({rc['speedup_vs_f32']:.2f}x), "
            f"fit {rc['fit_error']:.4e}")
        torch.cuda.empty_cache()
    del X64
    extra = {}
    for key in [k for k in args.forms.split(",") if k and k != args.config]:
        form, Xf, initf, cfgf = workload_form(args, key)
        out["forms"][cfgf["name"]] = form
        extra[key] = (Xf, initf, cfgf)
    if not args.no_method_forms:
        if "c2" in extra:
            Xm, initm, cfgm = extra["c2"]
        else:
            cfgm = dict(synth.CONFIGS["c2"])
            Xm, _, initm = synth.make_config("c2", dtype=np.float32)
        out["forms"]["methods"] = method_forms(args, Xm, initm, cfgm)
        del Xm
    extra.clear()
    torch.cuda.empty_cache()
    if not args.no_oscillatory_form:
        out["forms"]["oscillatory"] = oscillatory_form(args)
        torch.cuda.empty_cache()
    if not args.no_serving_form:
        out["forms"]["serving"] = serving_form(args)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(X, init, cfg, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
