"""Throughput of full Greek sets on one MI355X.

A step is one whole Greek set of the 10-asset Heston best-of American call
(200,000 paths x 252 steps, 78 bump-and-revalue scenarios with common random
numbers: base, 2 x 10 spot, 10 v0, maturity, rate and 45 correlation bumps;
FP32 paths / FP64 regression): path kernel, Gram kernel, backward sweep,
results back on the host, Greeks.  The launch shape is autotuned first and
each pass of the set replays a cached HIP graph.  Inputs are seeded and
synthetic and already in HBM; only the few-KB parameter tables go up and the
scenario prices come back.  The 5-asset 25,000 x 252 set (28 scenarios) is
timed after it as a secondary figure.

Printed: one JSON line with the metric (Greek-set path-steps/s; the median and
spread of the per-set times beside the mean), the roofline of the dominant
kernel (HIP-event times on the library's stream), the FP64 oracle timed on the
host cores (one thread and all cores) on a sample of whole scenarios, the
accuracy of the timed results against the oracle on those scenarios, the plain
per-scenario FP64 GPU comparator, and p50/p99 request latency of the serving
loop under a Poisson stream of mixed-size requests.  --serve-sweep instead
runs only the serving loop at offered loads 0.5, 0.8 and 0.95.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = "Greek-set path-steps/s at <=1e-4 rel err vs FP64; p50/p99 request latency"
HBM_PEAK_GBS = 8000.0
# non-packed VALU lane-op slots per second: 256 CUs x 64 lanes x 2.4 GHz
ALU_PEAK_OPS = 256 * 64 * 2.4e9
CSRC = os.path.join(ROOT, "paper_2206_03719_amd", "csrc")
COUNTERS = {10: os.path.join(ROOT, "profiles", "greekset_bestof10_200000x252_hbm_counters.txt"),
            5: os.path.join(ROOT, "profiles", "greekset_bestof5_25000x252_hbm_counters.txt")}
# device kernel names (prefixes) of the three stages
KERNEL_NAMES = {"paths": "k_paths", "gram": "k_gram", "sweep": "k_sweep_cluster"}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def per_scenario_models(w):
    """The bumped models of the Greek set, one per scenario, in the library's
    scenario order (for the plain per-scenario comparator)."""
    m, C, opt, b = w["model"], w["corr"], w["option"], w["bumps"]
    N = len(m["S0"])
    out = [(m, C, opt)]
    for sgn in (1.0, -1.0):
        for a in range(N):
            mm = dict(m)
            mm["S0"] = m["S0"].copy()
            mm["S0"][a] = m["S0"][a] * (1.0 + sgn * b["spot_rel"])
            out.append((mm, C, opt))
    for a in range(N):
        mm = dict(m)
        mm["v0"] = m["v0"].copy()
        mm["v0"][a] = m["v0"][a] * (1.0 + b["v0_rel"])
        out.append((mm, C, opt))
    out.append((m, C, dict(opt, T=opt["T"] - b["T_abs"])))
    out.append((dict(m, r=m["r"] + b["r_abs"]), C, opt))
    for i in range(N):
        for j in range(i + 1, N):
            CC = C.copy()
            CC[i, j] += b["corr_abs"]
            CC[j, i] += b["corr_abs"]
            out.append((m, CC, opt))
    return out


def path_kernel_slots(N, P, n, mask):
    """Algorithmic VALU slots of the path kernel for one Greek set.

    Per element (one path, step and asset): the random numbers cost about 70
    slots (half a Philox4x32-10 call, ten rounds of two 32-bit multiply pairs
    at quarter rate, plus one Box-Muller pair: log, sqrt, sin, cos) and are
    paid once per base element, since every scenario reuses them; one
    full-truncation Euler step with its correlation row costs 25 + (N+1)/2
    slots (two sqrt and one exp at quarter rate, ~13 other operations) and is
    paid for every element whose path differs from the base path: the base's
    N assets, plus the bumped asset for the v0 scenarios, the assets at and
    after the later asset of the pair for the correlation scenarios and all N
    for the maturity scenario.  Spot scenarios rescale one asset of the base
    path, and the rate scenario all of them by one factor e^{(r' - r) t} (the
    rate enters the log price only through its drift): 4 slots each."""
    own = N  # base
    scaled = 0
    if mask & 1:
        scaled += 2 * N
    if mask & 2:
        own += N              # each v0 bump changes only its own asset
    if mask & 4:
        own += N              # maturity: a new time step for every asset
    if mask & 8:
        scaled += 1           # rate: the base path's U times e^{(r' - r) t}
    if mask & 16:
        own += sum(N - j for j in range(1, N) for _ in range(j))  # rows j.. of L
    per_path_step = 70 * N + (25 + (N + 1) / 2) * own + 4 * scaled
    return per_path_step * P * n


def kernel_source_sha256():
    """SHA-256 over the device sources (hs_*.hip and the headers they include),
    in name order: the kernel version a counter summary was taken on."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


def read_counters(path):
    """HBM bytes per dispatch from the committed counter summary, or None when
    it is missing or was taken on another version of the kernel source."""
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    src = kernel_source_sha256()
    fields = dict(l.split(":", 1) for l in lines if ":" in l and not l.startswith(("#", " ")))
    if fields.get("kernel_source_sha256", "").strip() != src:
        return None
    ff = float(fields["fetch_scale"])
    wf = float(fields["write_scale"])
    out = {}
    for l in lines:
        if l.startswith("traffic "):
            # traffic <stage> fetch_kib=<x> write_kib=<y>
            parts = l.split()
            kv = dict(p.split("=") for p in parts[2:])
            out[parts[1]] = (float(kv["fetch_kib"]) * ff + float(kv["write_kib"]) * wf) * 1024.0
    return out


def greek_set_leg(hs, torch, w, steps, warmup, graph, autotune, counters_path):
    """Times `steps` whole Greek sets of workload w (after `warmup` untimed
    ones) and returns the figures: the mean over the bracketed run, the median
    and spread of the per-set times, per-kernel device times from HIP events
    on the library's stream (the same sets launched eagerly), and the roofline
    of the dominant kernel."""
    N, P, n = len(w["model"]["S0"]), w["n_paths"], w["n_steps"]
    S = hs.num_scenarios(N, w["bumps"]["mask"])
    nbytes = hs.workspace_bytes(w["model"], w["option"], P, n, w["bumps"], "fp32")
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()  # a non-null stream: graph replay needs one

    def step(timing=False):
        return hs.price_greeks(w["model"], w["corr"], w["option"], P, n, w["bumps"],
                               seed=w["seed"], precision="fp32", workspace=ws, stream=stream,
                               timing=timing, graph=graph and not timing)

    tuned = None
    if autotune:
        tuned = hs.autotune(w["model"], w["corr"], w["option"], P, n, w["bumps"], seed=w["seed"],
                            workspace=ws, stream=stream, repeats=3, graph=graph)
        log("%s: autotuned, %.3f ms per Greek set" % (w["name"], tuned))
    log("%s: warmup %d" % (w["name"], warmup))
    for _ in range(warmup):
        res = step()
    torch.cuda.synchronize()
    log("%s: timing %d Greek sets%s" % (w["name"], steps, " (graph replay)" if graph else ""))
    per = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ta = time.perf_counter()
        res = step()  # returns with the results on the host (stream synchronized)
        per.append((time.perf_counter() - ta) * 1e3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / steps
    path_steps = S * P * n
    value = path_steps / (ms * 1e-3)
    log("%s: %.3f ms per Greek set (median %.3f), %.3e path-steps/s"
        % (w["name"], ms, float(np.median(per)), value))

    # per-kernel device times: the same sets launched eagerly with HIP events
    # around each stage on the library's stream
    kt = {"paths": [], "gram": [], "sweep": []}
    t0 = time.perf_counter()
    for _ in range(steps):
        r = step(timing=True)
        kt["paths"].append(r["t_paths_ms"])
        kt["gram"].append(r["t_gram_ms"])
        kt["sweep"].append(r["t_sweep_ms"])
    torch.cuda.synchronize()
    ms_eager = (time.perf_counter() - t0) * 1e3 / steps
    kms = {k: float(np.mean(v)) for k, v in kt.items()}
    log("%s: kernel ms (mean of %d): %s; eager set %.3f ms"
        % (w["name"], steps, json.dumps(kms), ms_eager))
    # algorithmic bytes per launch: features are 8 B (FP32 U, A) per path-step;
    # the path kernel writes them once, the Gram kernel reads dates 1..n-1,
    # the sweep reads every date once
    alg = {"paths": S * P * n * 8.0, "gram": S * P * (n - 1) * 8.0, "sweep": S * P * n * 8.0}
    slots = path_kernel_slots(N, P, n, w["bumps"]["mask"])
    traffic = read_counters(counters_path)
    per_kernel = {}
    for k in kms:
        sec = kms[k] * 1e-3
        per_kernel[k] = {"kernel": KERNEL_NAMES[k], "ms": round(kms[k], 4),
                         "alg_bytes": alg[k], "hbm_GBs": round(alg[k] / sec / 1e9, 1),
                         "hbm_frac": round(alg[k] / sec / 1e9 / HBM_PEAK_GBS, 4),
                         "traffic_bytes": traffic.get(k) if traffic else None}
    per_kernel["paths"]["alu_slots"] = slots
    per_kernel["paths"]["alu_frac"] = round(slots / (kms["paths"] * 1e-3) / ALU_PEAK_OPS, 4)
    dom = max(kms, key=kms.get)
    sec = kms[dom] * 1e-3
    if dom == "paths":
        # the path kernel is bound by VALU and transcendental issue, not HBM
        roofline = {"bound": "alu", "kernel": KERNEL_NAMES[dom],
                    "achieved": round(slots / sec / 1e12, 3), "peak": ALU_PEAK_OPS / 1e12,
                    "unit": "Tslot/s", "frac": round(slots / sec / ALU_PEAK_OPS, 4)}
    else:
        achieved = alg[dom] / sec / 1e9
        roofline = {"bound": "hbm", "kernel": KERNEL_NAMES[dom], "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4)}
    roofline["traffic"] = traffic.get(dom) if traffic else None
    roofline["kernel_ms"] = round(kms[dom], 4)
    roofline["per_kernel"] = per_kernel
    spread = {"median_ms": float(np.median(per)), "min_ms": float(np.min(per)),
              "max_ms": float(np.max(per)), "p10_ms": float(np.percentile(per, 10)),
              "p90_ms": float(np.percentile(per, 90)), "stdev_ms": float(np.std(per, ddof=1))
              if len(per) > 1 else 0.0, "sets": len(per),
              "median_path_steps_per_s": path_steps / (float(np.median(per)) * 1e-3)}
    del ws
    return {"value": value, "ms": ms, "spread": spread, "kernel_ms": kms, "eager_ms": ms_eager,
            "roofline": roofline, "res": res, "S": S, "path_steps": path_steps,
            "autotuned_ms": tuned, "stream": stream}


def cpu_baseline_leg(w, scen, threads_all, res):
    """The FP64 oracle on the host cores over whole scenarios of the Greek set
    (the regression couples all paths of a scenario, so a prefix of paths would
    be another problem): the scenarios `scen` at all cores, and the first of
    them at one thread.  Also the accuracy of the GPU's timed prices on them."""
    import oracle
    N, P, n = len(w["model"]["S0"]), w["n_paths"], w["n_steps"]
    nob = dict(w["bumps"], mask=0)
    models = per_scenario_models(w)
    out = {}
    prices = {}
    for label, threads, ss in (("all", threads_all, scen), ("one", 1, scen[:1])):
        log("cpu baseline: FP64 oracle, %d scenario(s) of %d x %d x %d, %d thread(s)"
            % (len(ss), N, P, n, threads))
        t0 = time.perf_counter()
        for s in ss:
            m, C, opt = models[s]
            prices[s] = oracle.price_greeks(m, C, opt, P, n, nob, w["seed"],
                                            nthreads=threads)["price"]
        sec = time.perf_counter() - t0
        out[label] = {"value": len(ss) * P * n / sec, "seconds": sec, "threads": threads,
                      "scenarios": list(ss)}
    err = {s: abs(res["scenario_price"][s] - p) / abs(p) for s, p in prices.items()}
    return out, {"max_price_rel_err": max(err.values()), "scenarios_checked": sorted(err)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-comparator", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--workload", choices=("bestof10", "bestof5"), default="bestof10")
    ap.add_argument("--serve-requests", type=int, default=300)
    ap.add_argument("--serve-slots", type=int, default=8,
                    help="requests the serving loop runs at once")
    ap.add_argument("--serve-sweep", action="store_true",
                    help="only the serving loop: --serve-requests (default 1000 here) requests "
                         "at offered loads 0.5, 0.8 and 0.95 of the saturated capacity")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device-to-device 5 times (HBM counter calibration)")
    ap.add_argument("--table1", action="store_true",
                    help="instead of the Greek set: the paper's Table 1 problem sizes through "
                         "the base-model path kernel, one JSON line per size and variant")
    ap.add_argument("--table1-sizes", default="tiny,small,medium,large,huge")
    ap.add_argument("--table1-variants", default="fp32:euler,fp64:euler,fp32:qe,fp64:qe")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs on a single MI355X and has no "
              "multi-GPU path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2206_03719_amd as hs

    hs.lib()
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied 1 GiB 5 times")
        return
    if args.table1:
        table1_leg(hs, torch, args)
        return
    if args.serve_sweep:
        n_req = args.serve_requests if "--serve-requests" in sys.argv else 1000
        for line in serve_sweep(hs, torch, n_req, args.serve_slots):
            print(json.dumps(line), flush=True)
        return
    graph = not args.no_graph
    if args.workload == "bestof10":
        w = W.best_of_call(n_assets=10, n_paths=200_000, n_steps=252, precision="fp32")
    else:
        w = W.best_of_call(n_assets=5, n_paths=25_000, n_steps=252, precision="fp32")
    N, P, n = len(w["model"]["S0"]), w["n_paths"], w["n_steps"]
    lg = greek_set_leg(hs, torch, w, args.steps, args.warmup, graph, not args.no_autotune,
                       COUNTERS[N])
    S, ms, value, res = lg["S"], lg["ms"], lg["value"], lg["res"]
    out = {"metric": METRIC, "value": value, "unit": "path-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "%s greek set (%d scenarios)" % (w["name"], S),
                      "n_assets": N, "n_paths": P, "n_steps": n, "n_scenarios": S,
                      "precision": "f32 paths, f64 regression", "seed": w["seed"],
                      "graph": graph, "autotuned": not args.no_autotune,
                      "elements_per_s": value * N, "eager_ms_per_step": lg["eager_ms"],
                      "autotune_best_ms": lg["autotuned_ms"]},
           "timing": lg["spread"],
           "roofline": lg["roofline"]}

    if not args.no_cpu_baseline:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        # base, spot up of asset 0, v0 of asset 0, correlation (0, 1) at all
        # cores; the base alone at one thread
        scen = [0, 1, 1 + 2 * N, 3 + 3 * N] if N > 1 else [0]
        cb, acc = cpu_baseline_leg(w, scen, threads, res)
        out["cpu_baseline"] = {"value": cb["all"]["value"], "unit": "path-steps/s",
                               "cores": threads, "kind": "oracle",
                               "sample": "scenarios %s of the set (base, spot up and v0 of "
                                         "asset 0, correlation (0, 1)), each whole: %d paths x "
                                         "%d steps in FP64; the regression couples all paths"
                                         % (scen, P, n),
                               "seconds": cb["all"]["seconds"], "cpu": cpu_model(),
                               "host_cpus": os.cpu_count(),
                               "one_thread": {"value": cb["one"]["value"],
                                              "seconds": cb["one"]["seconds"],
                                              "scenarios": cb["one"]["scenarios"]}}
        out["accuracy_vs_fp64_oracle"] = acc
        out["valid"] = bool(acc["max_price_rel_err"] <= 1e-4)
        log("accuracy: %s" % json.dumps(acc))

    if not args.no_comparator:
        log("comparator: plain per-scenario FP64 launches")
        models = per_scenario_models(w)
        nob = dict(w["bumps"], mask=0)
        wsb = max(hs.workspace_bytes(mm, oo, P, n, nob, "fp64") for mm, _, oo in models)
        ws64 = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        stream = lg["stream"]

        def plain():
            return [hs.price_greeks(mm, CC, oo, P, n, nob, seed=w["seed"], precision="fp64",
                                    workspace=ws64, stream=stream)["price"]
                    for mm, CC, oo in models]
        plain()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prices = plain()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        out["comparator_fp64_per_scenario"] = {
            "value": lg["path_steps"] / (t1 - t0), "unit": "path-steps/s",
            "ms": (t1 - t0) * 1e3, "speedup_of_batched": (t1 - t0) * 1e3 / ms,
            "max_rel_diff_vs_batched": float(np.max(np.abs(np.array(prices) -
                                                           res["scenario_price"]) /
                                                    np.abs(np.array(prices))))}
        del ws64
        log("comparator %.2f ms" % ((t1 - t0) * 1e3))

    if not args.no_secondary and args.workload == "bestof10":
        w5 = W.best_of_call(n_assets=5, n_paths=25_000, n_steps=252, precision="fp32")
        l5 = greek_set_leg(hs, torch, w5, max(args.steps, 10), args.warmup, graph, False,
                           COUNTERS[5])
        out["secondary"] = {"workload": "%s greek set (%d scenarios)" % (w5["name"], l5["S"]),
                            "value": l5["value"], "unit": "path-steps/s", "ms_per_step": l5["ms"],
                            "timing": l5["spread"], "kernel_ms": l5["kernel_ms"],
                            "roofline": {k: v for k, v in l5["roofline"].items()
                                         if k != "per_kernel"}}
        torch.cuda.empty_cache()

    if not args.no_serve:
        out["latency"] = serve_leg(hs, torch, args.serve_requests, 0.8, args.serve_slots)
        log("serving: %s" % json.dumps(out["latency"]))

    print(json.dumps(out), flush=True)


# The paper's multi-kernel runtimes (its Table A1: Heston paths plus the path
# reduction, FPGA and two 24-core CPUs, float and double), in ms.
PAPER_TA1_MS = {
    ("tiny", "float"): (46.11, 372.15), ("tiny", "double"): (75.97, 369.07),
    ("small", "float"): (82.01, 629.18), ("small", "double"): (141.39, 638.67),
    ("medium", "float"): (341.82, 1545.94), ("medium", "double"): (592.79, 1551.90),
    ("large", "float"): (1178.14, 4574.41), ("large", "double"): (1971.64, 4558.11),
    ("huge", "float"): (5838.23, 15825.42), ("huge", "double"): (10644.86, 15561.09),
}


def base_kernel_slots(N, P, n):
    """Algorithmic VALU slots of the base-model path kernel, FP32 Euler: per
    element the random numbers (about 70 slots, see path_kernel_slots) and one
    Euler step with its correlation row (25 + (N+1)/2 slots)."""
    return (70.0 + 25.0 + (N + 1) / 2.0) * N * P * n


def table1_leg(hs, torch, args):
    """The paper's Table 1 problem sizes (assets x daily steps x 25k paths)
    through hs_path_features: Heston paths and the per-date path reduction,
    the stage the paper times.  Device time of each call (model upload and
    kernel) from HIP events on the call's stream; elements = assets x steps x
    paths.  The FP64 oracle runs the same work on the host cores for the
    smallest size on a bounded sample of paths."""
    stream = torch.cuda.Stream()
    sizes = [s for s in args.table1_sizes.split(",") if s]
    variants = [tuple(v.split(":")) for v in args.table1_variants.split(",") if v]
    for size in sizes:
        w = W.paper_size(size)
        N, n, P, T = w["n_assets"], w["n_steps"], w["n_paths"], w["T"]
        elements = N * n * P
        for prec, scheme in variants:
            dt = torch.float32 if prec == "fp32" else torch.float64
            out = torch.empty((n, P, 2), dtype=dt, device="cuda")

            def call():
                with torch.cuda.stream(stream):
                    hs.path_features(w["model"], w["corr"], T, P, n, seed=w["seed"],
                                     precision=prec, scheme=scheme, stream=stream, out=out)
            for _ in range(max(1, args.warmup)):
                call()
            times = []
            for _ in range(args.steps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                call()
                e1.record(stream)
                e1.synchronize()
                times.append(e0.elapsed_time(e1))
            ms = float(np.median(times))
            fpga_ms, cpu_ms = PAPER_TA1_MS[(size, "float" if prec == "fp32" else "double")]
            line = {"table1": size, "n_assets": N, "n_steps": n, "n_paths": P, "T": T,
                    "precision": prec, "scheme": scheme, "ms": round(ms, 4),
                    "ms_min": round(float(np.min(times)), 4), "reps": args.steps,
                    "elements": elements, "elements_per_s": elements / (ms * 1e-3),
                    "paper_fpga_ms": fpga_ms, "paper_cpu_ms": cpu_ms,
                    "paper_fpga_elements_per_s": elements / (fpga_ms * 1e-3),
                    "x_paper_fpga": round(fpga_ms / ms, 1), "x_paper_cpu": round(cpu_ms / ms, 1)}
            if prec == "fp32" and scheme == "euler":
                slots = base_kernel_slots(N, P, n)
                line["alu_frac"] = round(slots / (ms * 1e-3) / ALU_PEAK_OPS, 4)
            log("%s %s %s: %.3f ms, %.3e elements/s (paper FPGA %.1f ms)"
                % (size, prec, scheme, ms, elements / (ms * 1e-3), fpga_ms))
            print(json.dumps(line), flush=True)
            del out
    if not args.no_cpu_baseline:
        import oracle
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        w = W.paper_size("tiny", n_paths=5000)
        N, n, P, T = w["n_assets"], w["n_steps"], w["n_paths"], w["T"]
        for scheme in ("euler", "qe"):
            t0 = time.perf_counter()
            oracle.features(w["model"], w["corr"], T, n, P, w["seed"], nthreads=threads,
                            scheme=scheme)
            sec = time.perf_counter() - t0
            print(json.dumps({"table1_cpu_baseline": "tiny", "scheme": scheme, "kind": "oracle",
                              "sample": "the first 5,000 of the 25,000 paths",
                              "elements_per_s": N * n * P / sec, "seconds": sec,
                              "cores": threads, "cpu": cpu_model()}), flush=True)


def cpu_model():
    try:
        for l in open("/proc/cpuinfo"):
            if l.startswith("model name"):
                return l.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _saturated(hs, srv, n_req):
    """All requests queued at once: requests/s and path-steps/s at saturation."""
    reqs = [r for _, r in W.serving_stream(n_req, 1.0, seed=11)]
    t0 = time.perf_counter()
    tickets = [srv.submit(r) for r in reqs]
    done = {}
    while len(done) < len(tickets):
        for t in tickets:
            if t not in done:
                p = srv.poll(t)
                if p is not None:
                    done[t] = p
                    if len(done) % 100 == 0:
                        log("saturated: %d of %d requests done" % (len(done), len(tickets)))
        time.sleep(0.001)
    t_sat = time.perf_counter() - t0
    steps = sum(hs.num_scenarios(len(r["model"]["S0"]), 31) * r["n_paths"] * r["n_steps"]
                for r in reqs)
    return len(reqs) / t_sat, steps / t_sat


def _poisson_run(hs, srv, n_req, rate, seed):
    """A Poisson stream of n_req requests at `rate` per second: latency from
    submit to result of each, and the path-steps/s the run sustained."""
    stream = W.serving_stream(n_req, rate, seed=seed)
    lat = []
    t0 = time.perf_counter()
    pending = {}
    i = 0
    while i < len(stream) or pending:
        now = time.perf_counter() - t0
        while i < len(stream) and stream[i][0] <= now:
            pending[srv.submit(stream[i][1])] = True
            i += 1
        for t in list(pending):
            p = srv.poll(t)
            if p is not None:
                lat.append(p[1])
                del pending[t]
                if len(lat) % 100 == 0:
                    log("poisson stream at %.2f requests/s: %d of %d done"
                        % (rate, len(lat), len(stream)))
        time.sleep(0.0005)
    t_run = time.perf_counter() - t0
    steps = sum(hs.num_scenarios(len(r["model"]["S0"]), 31) * r["n_paths"] * r["n_steps"]
                for _, r in stream)
    lat = np.array(lat) * 1e3
    return {"requests": len(stream), "offered_req_per_s": rate,
            "path_steps_per_s": steps / t_run, "p50_ms": float(np.percentile(lat, 50)),
            "p90_ms": float(np.percentile(lat, 90)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max()), "seconds": t_run}


def _server(hs, torch, slots=8):
    free, total = torch.cuda.mem_get_info()
    pool = int(min(free * 0.7, 160e9))
    return hs.Server(pool, max_slots=slots), pool


def serve_leg(hs, torch, n_req, load, slots=8):
    """Poisson stream of mixed-size full-Greek-set requests (assets U{1..20},
    paths U[10k, 400k], steps U{52,126,252,504}) through the serving loop.
    First the saturated capacity (all requests queued at once), then a
    Poisson stream at `load` of it: p50/p99 latency from submit to result."""
    srv, pool = _server(hs, torch, slots)
    try:
        cap, sat_steps = _saturated(hs, srv, n_req)
        run = _poisson_run(hs, srv, n_req, load * cap, seed=12)
        st = srv.stats()
        return dict(run, offered_load=load, saturated_req_per_s=cap,
                    saturated_path_steps_per_s=sat_steps, pool_GB=pool / 1e9,
                    pool_peak_GB=st["pool_peak"] / 1e9, slots=st["slots"],
                    device_max_concurrent=st["device_max_concurrent"],
                    device_overlap_s=st["device_overlap_s"])
    finally:
        srv.close()


def serve_sweep(hs, torch, n_req, slots=8):
    """The serving loop at offered loads 0.5, 0.8 and 0.95 of its saturated
    capacity, n_req requests each: one JSON line per load."""
    srv, pool = _server(hs, torch, slots)
    try:
        log("serve sweep: saturated capacity over %d requests" % n_req)
        cap, sat_steps = _saturated(hs, srv, n_req)
        log("serve sweep: %.2f requests/s, %.3e path-steps/s saturated" % (cap, sat_steps))
        out = []
        for i, load in enumerate((0.5, 0.8, 0.95)):
            log("serve sweep: offered load %.2f" % load)
            run = _poisson_run(hs, srv, n_req, load * cap, seed=20 + i)
            line = dict(run, serve_sweep=True, offered_load=load, saturated_req_per_s=cap,
                        saturated_path_steps_per_s=sat_steps, pool_GB=pool / 1e9)
            log(json.dumps(line))
            out.append(line)
        st = srv.stats()
        out.append({"serve_sweep_stats": st})
        return out
    finally:
        srv.close()


if __name__ == "__main__":
    main()
