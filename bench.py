#!/usr/bin/env python3
"""Benchmark of the string sample sort on one MI355X.

One step = one complete sort (permutation + LCP array) of the 16M-string
Markov workload (lognormal lengths, median 40, order-2 Markov chain over 64
symbols with Zipf(1.1) transitions, ~0.8 GB of characters), inputs resident
in HBM.  Prints ONE JSON line on stdout; details go to stderr.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--workload NAME]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sorted chars/s + strings/s incl. LCP, %HBM peak; batched vs per-set launch"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per work unit of each kernel (what the kernel must move
# by its definition, not what the hardware ends up fetching).
#   k_init      per string: offset (8) + first word (<= 8, measured) + record write (13)
#   k_classify  per string: key and r read (9) + bucket id write (2)
#   k_scatter   per string and distribution pass: 2 x 13 (read + write of
#               idx u32, key u64, r u8), the byte model of one distribution pass
#   k_base      per string: record read (13) + perm and lcp writes (4 + 4)
#   k_scan      per counter: reduce read (4) + scan read (4) + write (4)
#   k_lcp_fill  per boundary: entry (8) + lcp (4+4) + perm (8) + offsets (32) + two words (16)
# The implementation's records are 16 bytes (key, idx, len) and the scatter
# also reads the 2-byte bucket id, 34 bytes per string; that figure is
# reported beside the model's 26.
BYTES_PER_UNIT = {
    "k_classify": 11.0,
    "k_scatter": 26.0,
    "k_base": 21.0,
    "k_base_wave1": 21.0,
    "k_base_wave2": 21.0,
    "k_base_wave4": 21.0,
    "k_scan": 12.0,
    "k_lcp_fill": 72.0,
}
SCATTER_IMPL_BYTES = 34.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the sort kernels' sources with comments and blank space
    removed (a comment edit does not change the code the counters saw)."""
    import re
    h = hashlib.sha256()
    for f in ("ss_kernels.hip", "ss_device.h", "ss_gather.h", "ss_internal.h"):
        with open(os.path.join(ROOT, "paper_1808_00963_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources and on this workload; else
    None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash() or t.get("workload") != workload:
        return None
    k = t.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k.get("bytes_per_launch")


def event_ms(fn, reps, stream):
    """Median milliseconds of fn() over reps runs, HIP events on `stream`
    around each run (one warm-up run first)."""
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def wall_ms(fn, reps):
    """Median wall milliseconds of fn() with the device synchronised around
    each run (one warm-up run first)."""
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        a = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - a) * 1e3)
    ts.sort()
    return ts[len(ts) // 2]


def batch_measure(steps, sets=4096, autotune=False):
    """Batched workload: `sets` independent sets (character budgets
    log-uniform in [1e3, 1e6], model per set uniform over the four
    generators).  Times a loop of per-set ss_sort_ex calls on one stream
    against the batched forms (device-driven levels, host-driven levels, one
    persistent launch, the hipGraph); all forms must give identical
    outputs.  Wall time with the device synchronised around each run."""
    import ctypes

    import numpy as np
    import torch

    import gen
    import paper_1808_00963_amd as ss

    t0 = time.perf_counter()
    c, o, sb = gen.batch_sets(num_sets=sets)
    n, N, S = len(o) - 1, int(o[-1]), len(sb) - 1
    log(f"batched workload: {S} sets, n={n} N={N} ({time.perf_counter() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    chars = torch.from_numpy(c).to(dev)
    offs = torch.from_numpy(o.view(np.int64)).to(dev)
    sbd = torch.from_numpy(sb.astype(np.int32)).to(dev)
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    ctx = ss.Context(0)
    lib = ss.lib()
    outs = {}
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    lcp = torch.empty(n, dtype=torch.int32, device=dev)
    cp, op, pp, lp = chars.data_ptr(), offs.data_ptr(), perm.data_ptr(), lcp.data_ptr()
    bounds = [(int(sb[j]), int(sb[j + 1])) for j in range(S)]

    def per_set():
        for b, e in bounds:
            st = lib.ss_sort_ex(ctx._h, ctypes.c_void_p(cp), ctypes.c_void_p(op + 8 * b), e - b,
                                ctypes.c_void_p(pp + 4 * b), ctypes.c_void_p(lp + 4 * b), sp)
            if st:
                raise ss.SSError(st, "ss_sort_ex")

    ms = {}
    ctx.set_config(mode="levels")
    ms["per_set_launches"] = wall_ms(per_set, 1)
    outs["per_set_launches"] = (perm.clone(), lcp.clone())
    for form, mode in (("batched_levels", "levels"), ("batched_host_levels", "host_levels"),
                       ("batched_persistent", "persistent")):
        ctx.set_config(mode=mode)
        ms[form] = wall_ms(lambda: ctx.sort_batch(chars, offs, sbd, perm, lcp, stream), steps)
        outs[form] = (perm.clone(), lcp.clone())
    ctx.set_config(mode="levels")
    g = ctx.graph_batch(chars, offs, sbd, perm, lcp)

    def graph_run():
        g.launch(stream)

    ms["batched_graph"] = wall_ms(graph_run, steps)
    ctx.sync(stream)
    outs["batched_graph"] = (perm.clone(), lcp.clone())
    graph_levels = g.levels
    g.close()
    tune = None
    if autotune:
        tctx = ss.Context(0)
        t_a = time.perf_counter()
        tuned_cfg, tuned_ms, _, _ = tctx.autotune(chars, offs, sbd, perm, lcp, reps=2, stream=stream)
        tune_s = time.perf_counter() - t_a
        ms["batched_autotuned"] = wall_ms(lambda: tctx.sort_batch(chars, offs, sbd, perm, lcp, stream), steps)
        outs["batched_autotuned"] = (perm.clone(), lcp.clone())
        tune = {"config": tuned_cfg, "tuner_median_ms": tuned_ms, "tuning_s": tune_s}
    ref = outs["per_set_launches"]
    identical = all(torch.equal(v[0], ref[0]) and torch.equal(v[1], ref[1]) for v in outs.values())
    for k, v in ms.items():
        log(f"{k:22s} {v:9.3f} ms  {N / v / 1e6:8.2f} G chars/s")
    forms = [k for k in ms if k != "per_set_launches"]
    best = min(forms, key=lambda k: ms[k])
    del chars, offs, sbd, perm, lcp, outs
    torch.cuda.empty_cache()
    return {"sets": S, "n_strings": n, "n_chars": N, "ms": ms, "best_form": best,
            "graph_level_launches": graph_levels,
            "graph_vs_per_set": ms["per_set_launches"] / ms["batched_graph"],
            "best_vs_per_set": ms["per_set_launches"] / ms[best],
            "outputs_identical": identical, "autotune": tune}


def run_batch(args):
    r = batch_measure(args.steps, sets=args.sets, autotune=True)
    best = r["best_form"]
    out = {
        "metric": METRIC, "value": r["n_chars"] / (r["ms"][best] * 1e-3), "unit": "chars/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": r["ms"][best], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "batched_4096_sets", "sets": r["sets"], "n_strings": r["n_strings"],
                   "n_chars": r["n_chars"], "form": best},
        "batched_vs_per_set": r["best_vs_per_set"], **r,
    }
    print(json.dumps(out), flush=True)


def serve_measure(pool_size=128, requests=2000, warmup=200, check=8):
    """Serving workload: a Poisson stream of sort requests, sizes
    log-uniform in [1e3, 1e6] strings from the Markov generator, admitted by
    an 8 GB HBM budget.  Saturation throughput mu is measured closed-loop
    first; open-loop runs at 0.5 mu and 0.8 mu report p50/p99 latency
    (submit -> outputs on the host) and chars/s.  Requests cycle through a
    pool of distinct pre-generated requests in pinned host memory.  After
    the timed runs, `check` completed requests of the pool are verified
    against the oracle (outside the timed region)."""
    import threading

    import numpy as np
    import torch

    import gen
    import paper_1808_00963_amd as ss

    seed, P = 6, pool_size
    t0 = time.perf_counter()
    pool = []
    for j in range(P):
        nj = gen.log_uniform(seed, j, 1e3, 1e6)
        c, o = gen.generate("markov", nj, gen.mix(seed, j))
        cp = torch.empty(len(c), dtype=torch.uint8, pin_memory=True).numpy()
        cp[:] = c
        op = torch.empty(len(o) * 8, dtype=torch.uint8, pin_memory=True).numpy().view(np.uint64)
        op[:] = o
        pool.append((cp, op))
    sizes = np.array([len(o) - 1 for _, o in pool])
    # pinned result buffers per pool entry for the open-loop runs (at most a
    # few dozen requests are in flight there, so entries j and j + P never
    # overlap)
    outs = [tuple(torch.empty(max(int(n), 1) * 4, dtype=torch.uint8, pin_memory=True).numpy().view(np.uint32)
                  for _ in range(2)) for n in sizes]
    chars_of = np.array([int(o[-1]) for _, o in pool])
    log(f"serving pool: {P} requests, mean {sizes.mean():.0f} strings / {chars_of.mean() / 1e6:.2f} MB "
        f"({time.perf_counter() - t0:.1f}s)")
    srv = ss.Server(8 << 30, max_inflight=4096)
    for j in range(min(P, 32)):
        srv.wait(srv.submit(*pool[j]))
    srv.reset_stats()
    a = time.perf_counter()
    tickets = [srv.submit(*pool[j % P]) for j in range(min(requests, 600))]
    for t in tickets:
        srv.wait(t)
    dt = time.perf_counter() - a
    mu = len(tickets) / dt
    sat = srv.stats()
    log(f"saturation: {mu:.1f} req/s, {sat['chars_completed'] / dt / 1e9:.2f} G chars/s, "
        f"inflight_max {sat['inflight_max']}")

    def open_loop(rate, n_req, warm):
        srv.reset_stats()
        arrivals = np.cumsum([gen.exponential(seed + 1, j) / rate for j in range(n_req)])
        tickets = [None] * n_req
        lats = [None] * n_req
        start = time.perf_counter() + 0.05

        def submitter():
            for j in range(n_req):
                d = start + arrivals[j] - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tickets[j] = (srv.submit(*pool[j % P], *outs[j % P]), time.perf_counter())

        th = threading.Thread(target=submitter)
        th.start()
        done_chars = 0
        t_first = None
        for j in range(n_req):
            while tickets[j] is None:
                time.sleep(0.0002)
            _, _, lat = srv.wait(tickets[j][0])
            lats[j] = lat
            if j == warm:
                t_first = time.perf_counter()
            if j >= warm:
                done_chars += int(chars_of[j % P])
        th.join()
        t_end = time.perf_counter()
        L = np.array(lats[warm:]) / 1e3
        st = srv.stats()
        # the slowest requests: index, strings, latency, submission time
        # from the first measured request (for reading the tail)
        worst = np.argsort(L)[::-1][:12]
        tail = [[int(warm + q), int(sizes[(warm + q) % P]), round(float(L[q]), 3),
                 round(float(arrivals[warm + q] - arrivals[warm]) * 1e3, 2)] for q in worst]
        return {"rate_req_s": rate, "requests": n_req - warm, "p50_ms": float(np.percentile(L, 50)),
                "p99_ms": float(np.percentile(L, 99)), "mean_ms": float(L.mean()),
                "chars_per_s": done_chars / (t_end - t_first), "inflight_max": st["inflight_max"],
                "footprint_max_gb": st["footprint_max"] / 1e9,
                "iter_max_ms": st["iter_max_us"] / 1e3, "iter_max_wait_ms": st["iter_max_wait_us"] / 1e3,
                "iter_max_stage_ms": st["iter_max_stage_us"] / 1e3,
                "slowest": {"columns": ["request", "strings", "latency_ms", "arrival_ms"], "rows": tail}}

    res = {}
    for frac in (0.5, 0.8):
        r = open_loop(frac * mu, requests + warmup, warmup)
        res[str(frac)] = r
        log(f"rate {frac:.1f} mu = {r['rate_req_s']:.1f} req/s: p50 {r['p50_ms']:.2f} ms, p99 "
            f"{r['p99_ms']:.2f} ms, {r['chars_per_s'] / 1e9:.2f} G chars/s, inflight_max {r['inflight_max']}")
    # results checked outside the timed runs: a spread of pool requests,
    # submitted together, each against the oracle's definition
    import oracle
    idx = sorted(range(P), key=lambda j: sizes[j])[:: max(1, P // check)][:check]
    tk = [srv.submit(*pool[j]) for j in idx]
    fails = []
    for j, t in zip(idx, tk):
        p, l, _ = srv.wait(t)
        code = oracle.check(pool[j][0], pool[j][1], p, l)
        if code != -1:
            fails.append(f"request {j}: {oracle.describe_check(code, int(sizes[j]))}")
    srv.close()
    log(f"serving results checked against the oracle: {len(idx)} requests, {len(fails)} failures")
    return {"saturation_req_s": mu, "saturation_chars_per_s": sat["chars_completed"] / dt,
            "open_loop": res, "pool": P, "mean_strings": float(sizes.mean()),
            "checked_requests": len(idx), "check_failures": fails}


def run_serve(args):
    r = serve_measure(args.pool, args.requests, args.serve_warmup)
    main_r = r["open_loop"]["0.8"]
    out = {
        "metric": METRIC, "value": main_r["chars_per_s"], "unit": "chars/s", "n_gpus": 1,
        "steps": main_r["requests"], "warmup": args.serve_warmup, "ms_per_step": main_r["mean_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "serving_poisson_markov", "budget_bytes": 8 << 30, "pool": args.pool,
                   "sizes": "log-uniform 1e3..1e6 strings", "rate": "0.8 x saturation"},
        "p50_ms": main_r["p50_ms"], "p99_ms": main_r["p99_ms"], **r,
    }
    print(json.dumps(out), flush=True)


def run_merge(args):
    """LCP-aware merge of K sorted runs: the workload's strings are cut into
    K contiguous runs, sorted by the batched sort (untimed set-up), and the
    timed step is one ss_merge_runs of the K runs into one sorted sequence
    with its LCP array."""
    import numpy as np
    import torch

    import gen
    import paper_1808_00963_amd as ss

    model, n, seed = gen.WORKLOADS[args.workload]
    c, o = gen.generate(model, n, seed)
    N = int(o[-1])
    dev = torch.device("cuda:0")
    chars = torch.from_numpy(c).to(dev)
    offs = torch.from_numpy(o.view(np.int64)).to(dev)
    K = max(1, args.runs)
    rb = [n * r // K for r in range(K + 1)]
    ctx = ss.Context(0)
    sb = torch.tensor(rb, dtype=torch.int32, device=dev)
    p, l = ctx.sort_batch(chars, offs, sb)
    for r in range(K):  # set-local -> global string indices
        p[rb[r]:rb[r + 1]] += rb[r]
    mp = torch.empty(n, dtype=torch.int32, device=dev)
    ml = torch.empty(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        ctx.merge_runs(chars, offs, p, l, rb, mp, ml, stream=stream)
    ctx.set_profiling(True)
    ctx.reset_kernel_times()
    for _ in range(args.steps):
        ctx.merge_runs(chars, offs, p, l, rb, mp, ml, stream=stream)
    torch.cuda.synchronize()
    ctx.set_profiling(False)
    kt = ctx.kernel_times()
    dom = "k_merge_tile"
    ctx.set_profiling(True, only=dom)
    ctx.reset_kernel_times()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.merge_runs(chars, offs, p, l, rb, mp, ml, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.set_profiling(False)
    d = ctx.kernel_times()[dom]
    sec = (t1 - t0) / args.steps
    # k_merge_tile per string and round: perm + lcp in (8) and out (8), the
    # string's offset pair (16) and one 8-byte word of its characters (8);
    # the last two are random accesses (a 64-byte HBM burst each)
    alg = d["units"] / d["launches"] * 40.0
    avg_ms = d["total_ms"] / d["launches"]
    achieved = alg / (avg_ms * 1e-3) / 1e9
    for k, v in sorted(kt.items(), key=lambda kv: -kv[1]["total_ms"]):
        if v["launches"]:
            print(f"[bench] {k:14s} {v['total_ms'] / args.steps:8.3f} ms/step  launches/step "
                  f"{v['launches'] / args.steps:5.1f}", file=sys.stderr)
    # context: a full sort of the same strings
    ctx.sort(chars, offs, mp, ml)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(args.steps):
        ctx.sort(chars, offs, mp, ml)
    torch.cuda.synchronize()
    sort_ms = (time.perf_counter() - a) / args.steps * 1e3
    print(f"[bench] merge of {K} runs {sec * 1e3:.3f} ms, full sort {sort_ms:.3f} ms", file=sys.stderr, flush=True)
    # CPU baseline: the oracle's answer for a merge is its sort of the union
    # (the result is unique); timed on a bounded prefix of the workload
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        ns = min(n, args.cpu_sample if args.cpu_sample > 0 else 1 << 21)
        a = time.perf_counter()
        oracle.sort(c[: int(o[ns])], o[: ns + 1])
        dt = time.perf_counter() - a
        cpu = {"value": ns / dt, "unit": "strings/s", "cores": 1, "kind": "oracle",
               "sample": f"oracle sort of the first {ns} strings of {args.workload} (the merge's unique result), "
                         f"qsort+memcmp and brute LCP, 1 thread, {dt:.2f} s"}
    print(json.dumps({
        "metric": "merged strings/s (LCP-aware merge of K sorted runs, perm + LCP)", "value": n / sec,
        "unit": "strings/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": args.workload, "model": model, "n_strings": n, "n_chars": N, "runs": K,
                   "parallelism": "single-gpu"},
        "chars_per_s": N / sec, "full_sort_ms": sort_ms, "cpu_baseline": cpu,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "alg_bytes_per_launch": alg,
                     "avg_launch_ms": avg_ms},
        "kernel_ms_per_step": {k: v["total_ms"] / args.steps for k, v in kt.items() if v["launches"]},
    }), flush=True)


def run_sa(args):
    """Suffix array by prefix doubling of a seeded ACGT text with planted
    1 KiB repeats (the text of the suffix workload), 2^24 characters by
    default (--sa-n); one step = one complete ss_suffix_array call."""
    import numpy as np
    import torch

    import gen
    import paper_1808_00963_amd as ss

    n = args.sa_n
    t = gen.text("dna", n, 4)
    text = torch.from_numpy(t).cuda()
    sa = torch.empty(n, dtype=torch.int32, device="cuda")
    isa = torch.empty_like(sa)
    ctx = ss.Context(0)
    stream = torch.cuda.current_stream()
    rounds = 0
    for _ in range(args.warmup):
        _, _, rounds = ctx.suffix_array(text, sa, isa, stream=stream)
    ctx.set_profiling(True)
    ctx.reset_kernel_times()
    for _ in range(args.steps):
        ctx.suffix_array(text, sa, isa, stream=stream)
    torch.cuda.synchronize()
    ctx.set_profiling(False)
    kt = ctx.kernel_times()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, rounds = ctx.suffix_array(text, sa, isa, stream=stream)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    for k, v in sorted(kt.items(), key=lambda kv: -kv[1]["total_ms"]):
        if v["launches"]:
            print(f"[bench] {k:14s} {v['total_ms'] / args.steps:8.3f} ms/step  launches/step "
                  f"{v['launches'] / args.steps:5.1f}", file=sys.stderr)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        ns = min(n, args.cpu_sample if args.cpu_sample > 0 else 1 << 21)
        a = time.perf_counter()
        oracle.suffix_array(t[:ns])
        dt = time.perf_counter() - a
        cpu = {"value": ns / dt, "unit": "suffixes/s", "cores": 1, "kind": "oracle",
               "sample": f"suffix array of the first {ns} characters of the text, qsort of suffixes, 1 thread, "
                         f"{dt:.2f} s"}
    print(f"[bench] suffix array n={n}: {sec * 1e3:.3f} ms, {rounds} sorts", file=sys.stderr, flush=True)
    # roofline of the dominant kernel with known algorithmic bytes (the
    # sorter's), from the breakdown pass's HIP events
    roof = None
    known = [k for k in kt if k in BYTES_PER_UNIT and kt[k]["launches"]]
    if known:
        dom = max(known, key=lambda k: kt[k]["total_ms"])
        d = kt[dom]
        alg = d["units"] / d["launches"] * BYTES_PER_UNIT[dom]
        avg_ms = d["total_ms"] / d["launches"]
        ach = alg / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": None, "alg_bytes_per_launch": alg, "avg_launch_ms": avg_ms}
    print(json.dumps({
        "metric": "suffixes/s (suffix array by prefix doubling on the string sorter)", "value": n / sec,
        "unit": "suffixes/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"dna_text_{n}", "text": "ACGT, planted 1 KiB repeats", "n": n, "rounds": rounds,
                   "parallelism": "single-gpu"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernel_ms_per_step": {k: v["total_ms"] / args.steps for k, v in kt.items() if v["launches"]},
    }), flush=True)


def run_profile(args):
    """Program for hardware-counter runs: 3 streaming copies of 1 GiB (known
    traffic, for calibration) followed by warm-up + timed sorts of the plain
    workload.  Prints the copy bandwidth."""
    import numpy as np
    import torch

    import gen
    import paper_1808_00963_amd as ss

    nbytes = 1 << 30
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    torch.cuda.synchronize()
    ts = []
    for _ in range(3):
        a = time.perf_counter()
        ss.hbm_copy(dst, src)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - a)
    print(f"[bench] copy 1 GiB: {2 * nbytes / min(ts) / 1e9:.1f} GB/s (read + write)", file=sys.stderr, flush=True)
    del src, dst
    model, n, seed = gen.WORKLOADS[args.workload]
    c, o = gen.generate(model, n, seed)
    chars = torch.from_numpy(c).cuda()
    offs = torch.from_numpy(o.view(np.int64)).cuda()
    ctx = ss.Context(0)
    for _ in range(args.warmup):  # each finished before the next: the level budget follows the workload
        ctx.sort(chars, offs)
        ctx.sync()
    for _ in range(args.steps):
        ctx.sort(chars, offs)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "profile", "workload": args.workload, "copy_gbs": 2 * nbytes / min(ts) / 1e9}))


def run_traffic(args):
    """Turns two rocprofv3 counter runs of `--mode profile` (FETCH_SIZE, then
    WRITE_SIZE; KiB per dispatch) into calibrated HBM bytes per launch of
    every kernel of ONE sort, written to profiles/traffic.json (with the hash
    of the kernel sources it was taken on) and a text summary.  Calibration:
    the streaming copy moves exactly 1 GiB each way, so each counter's
    reading for it gives the factor that turns that counter into bytes."""
    import csv
    import numpy as np

    def per_dispatch(path, counter):
        rows = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                did = int(r["Dispatch_Id"])
                name = r["Kernel_Name"]
                rows.setdefault(did, [name, 0.0])
                rows[did][1] += float(r["Counter_Value"]) * 1024.0  # KiB -> bytes
        return [rows[k] for k in sorted(rows)]

    fetch = per_dispatch(args.fetch_csv, "FETCH_SIZE")
    write = per_dispatch(args.write_csv, "WRITE_SIZE")
    copy_bytes = 1 << 30
    calib = {}
    for tag, rows in (("fetch", fetch), ("write", write)):
        copies = [v for k, v in rows if "k_copy" in k]
        if not copies:
            raise SystemExit(f"no copy kernel dispatch in the {tag} run")
        calib[tag] = copy_bytes / float(np.median(copies))

    def last_sort(rows):
        starts = [i for i, (k, _) in enumerate(rows) if "k_reset" in k]
        return rows[starts[-1]:]

    def short(name):
        # library names: k_base_wave<E, AC> -> k_base_wave<E>, k_x<AC> -> k_x
        base = name.split("(")[0].replace("void ", "").replace("ss::", "")
        if "<" in base:
            kern, targs = base[:base.index("<")], base[base.index("<") + 1:].rstrip(">").split(",")
            base = f"k_base_wave{targs[0].strip()}" if kern == "k_base_wave" else kern
        return base

    kern = {}
    for (kf, vf), (kw, vw) in zip(last_sort(fetch), last_sort(write)):
        if short(kf) != short(kw):
            raise SystemExit("fetch and write runs dispatched different kernels")
        d = kern.setdefault(short(kf), {"launches": 0, "fetch": 0.0, "write": 0.0})
        d["launches"] += 1
        d["fetch"] += vf * calib["fetch"]
        d["write"] += vw * calib["write"]
    out = {"kernel_source_hash": kernel_source_hash(), "workload": args.workload,
           "calibration": {"copy_bytes_each_way": copy_bytes, "fetch_factor": calib["fetch"],
                           "write_factor": calib["write"]},
           "command_fetch": "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out> -o run -- "
                            "python3 bench.py --mode profile --steps 1 --warmup 1",
           "command_write": "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <out> -o run -- "
                            "python3 bench.py --mode profile --steps 1 --warmup 1",
           "kernels": {}}
    for k, d in kern.items():
        L = d["launches"]
        out["kernels"][k] = {"launches": L, "fetch_bytes_per_launch": d["fetch"] / L,
                             "write_bytes_per_launch": d["write"] / L,
                             "bytes_per_launch": (d["fetch"] + d["write"]) / L}
    # the whole sort as one entry (every kernel of one sort)
    tf = sum(d["fetch"] for d in kern.values())
    tw = sum(d["write"] for d in kern.values())
    out["kernels"]["__sort__"] = {"launches": 1, "fetch_bytes_per_launch": tf, "write_bytes_per_launch": tw,
                                  "bytes_per_launch": tf + tw}
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as f:
        json.dump(out, f, indent=1)
    lines = [f"# HBM traffic per kernel launch from hardware counters, one full sort of {args.workload}.",
             "# Commands (from /tmp, TMPDIR=/tmp), one counter per run:",
             f"#   {out['command_fetch']}", f"#   {out['command_write']}",
             "# then: python3 bench.py --mode traffic --fetch-csv <fetch csv> --write-csv <write csv>",
             f"# Calibration: ss_hbm_copy of 1 GiB each way; FETCH_SIZE factor {calib['fetch']:.3f}, "
             f"WRITE_SIZE factor {calib['write']:.3f} (bytes per counted byte).  Values are calibrated bytes.",
             "# Columns: kernel | launches per sort | fetch MB/launch | write MB/launch | total MB/launch", ""]
    for k, v in sorted(out["kernels"].items(), key=lambda kv: -kv[1]["bytes_per_launch"] * kv[1]["launches"]):
        lines.append(f"{k:14s} | {v['launches']:2d} | {v['fetch_bytes_per_launch'] / 1e6:9.1f} | "
                     f"{v['write_bytes_per_launch'] / 1e6:9.1f} | {v['bytes_per_launch'] / 1e6:9.1f}")
    with open(os.path.join(ROOT, "profiles", f"traffic_{args.workload}_pmc.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print(json.dumps({"mode": "traffic", "kernels": len(kern)}))


def run_counters(args):
    """Per-kernel sums of hardware counters over the last sort of a
    `--mode profile` run (rocprofv3 --pmc ... --output-format csv), one or
    more counter CSVs, written to profiles/counters_<workload>.txt with the
    per-wave figures (counter / SQ_WAVES) where SQ_WAVES was collected."""
    import csv

    per = {}   # dispatch id -> (kernel, {counter: value})
    for path in args.csv:
        with open(path) as f:
            for r in csv.DictReader(f):
                did = (path, int(r["Dispatch_Id"]))
                e = per.setdefault(did, [r["Kernel_Name"], {}])
                e[1][r["Counter_Name"]] = e[1].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    kern = {}
    counters = []
    for path in args.csv:
        rows = [per[k] for k in sorted(k for k in per if k[0] == path)]
        starts = [i for i, (name, _) in enumerate(rows) if "k_reset" in name]
        seen = set(counters)  # a counter collected in several runs is taken from the first
        for name, vals in rows[starts[-1]:] if starts else rows:
            base = name.split("(")[0].replace("void ", "").replace("ss::", "")
            d = kern.setdefault(base, {})
            for c, v in vals.items():
                if c in seen:
                    continue
                if c not in counters:
                    counters.append(c)
                d[c] = d.get(c, 0.0) + v
    lines = [f"# Hardware counters summed per kernel over one sort of {args.workload}.",
             "# Commands (from /tmp, TMPDIR=/tmp), one counter group per run:"]
    lines += [f"#   rocprofv3 --pmc {g} --output-format csv -d <out> -o run -- "
              "python3 bench.py --mode profile --steps 1 --warmup 1" for g in args.groups or []]
    lines += ["# then: python3 bench.py --mode counters --csv <csv> [--csv <csv> ...]",
              "# Rows: kernel; columns: counter totals (and per wave, /w, where SQ_WAVES was collected)", ""]
    hdr = f"{'kernel':16s}" + "".join(f" {c[:22]:>22s}" for c in counters)
    lines.append(hdr)
    order = sorted(kern, key=lambda k: -kern[k].get("SQ_WAVES", 0.0))
    for k in order:
        d = kern[k]
        cells = []
        for c in counters:
            v = d.get(c)
            if v is None:
                cells.append(f" {'-':>22s}")
            elif "SQ_WAVES" in d and c != "SQ_WAVES" and d["SQ_WAVES"] > 0:
                cells.append(f" {v:12.4g} {v / d['SQ_WAVES']:7.1f}/w")
            else:
                cells.append(f" {v:22.4g}")
        lines.append(f"{k[:16]:16s}" + "".join(cells))
    out = os.path.join(ROOT, "profiles", f"counters_{args.workload}.txt")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def run_stats(args):
    """Formats a rocprofv3 `--stats` kernel summary (kernel_stats.csv) of a
    bench.py run as profiles/kernels_<workload>_stats.txt; the bench line of
    the same run (--bench-json) adds its own event average of the dominant
    kernel for comparison."""
    import csv

    rows = []
    with open(args.csv[0]) as f:
        for r in csv.DictReader(f):
            rows.append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]) / 1e6, float(r["AverageNs"]) / 1e3,
                         float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    rows.sort(key=lambda x: -x[2])
    lines = [f"# rocprofv3 kernel statistics, {args.workload}, one MI355X.",
             "# Command (from /tmp, TMPDIR=/tmp):",
             f"#   rocprofv3 --kernel-trace --stats --output-format csv -d <out> -o run -- python3 bench.py {args.command}",
             f"# then: python3 bench.py --mode stats --workload {args.workload} --csv <kernel_stats.csv> "
             "--bench-json <the run's bench line>"]
    for note in args.note or []:
        lines.append(f"# {note}")
    if args.bench_json:
        with open(args.bench_json) as f:
            b = json.loads([ln for ln in f.read().splitlines() if ln.startswith("{")][-1])
        rf = b.get("roofline", {})
        if rf.get("avg_launch_ms"):
            lines.append(f"# bench.py's HIP-event average of {rf.get('kernel')} in the same run: "
                         f"{rf['avg_launch_ms'] * 1e3:.1f} us per launch; step {b['ms_per_step']:.3f} ms.")
    lines += ["", f"{'kernel':60s} {'calls':>6s} {'total ms':>9s} {'avg us':>8s} {'min us':>8s} {'max us':>8s} {'%':>6s}"]
    for name, calls, tot, avg, mn, mx, pct in rows:
        lines.append(f"{name[:60]:60s} {calls:6d} {tot:9.3f} {avg:8.1f} {mn:8.1f} {mx:8.1f} {pct:6.2f}")
    out = os.path.join(ROOT, "profiles", f"kernels_{args.workload}_stats.txt")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--mode", choices=["plain", "batch", "serve", "profile", "traffic", "counters", "stats", "merge", "sa"], default="plain")
    ap.add_argument("--fetch-csv", help="traffic mode: rocprofv3 counter_collection.csv of the FETCH_SIZE run")
    ap.add_argument("--write-csv", help="traffic mode: rocprofv3 counter_collection.csv of the WRITE_SIZE run")
    ap.add_argument("--csv", action="append", help="counters mode: a rocprofv3 counter_collection.csv")
    ap.add_argument("--groups", action="append", help="counters mode: the --pmc counter list of each run")
    ap.add_argument("--command", default="", help="stats mode: the bench.py arguments of the profiled run")
    ap.add_argument("--note", action="append", help="stats mode: a comment line for the summary")
    ap.add_argument("--bench-json", help="stats mode: the bench line printed by the profiled run")
    ap.add_argument("--pool", type=int, default=128)
    ap.add_argument("--runs", type=int, default=2, help="merge mode: number of sorted runs")
    ap.add_argument("--sa-n", type=int, default=1 << 24, help="sa mode: text length")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--sets", type=int, default=4096)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c1_markov_16m")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="plain mode: only the headline workload")
    ap.add_argument("--sort-mode", default="levels", choices=["levels", "host_levels", "persistent"],
                    help="how the recursion levels are driven (ss_config.mode)")
    ap.add_argument("--alphabet", default="bytes", choices=["auto", "bytes", "compress"],
                    help="key format (ss_config.alphabet): compressed keys where the input allows, or bytes")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="strings for the oracle timing (a prefix of the workload; 0 = all)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the sort runs on exactly one GPU (asked for {args.gpus}); "
              "sharding across GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)

    if args.mode == "batch":
        run_batch(args)
        return
    if args.mode == "serve":
        run_serve(args)
        return
    if args.mode == "profile":
        run_profile(args)
        return
    if args.mode == "traffic":
        run_traffic(args)
        return
    if args.mode == "counters":
        run_counters(args)
        return
    if args.mode == "stats":
        run_stats(args)
        return
    if args.mode == "merge":
        run_merge(args)
        return
    if args.mode == "sa":
        run_sa(args)
        return

    run_plain(args)


def alg_bytes(o, perm, lcp, dist_strings):
    """The byte model of the method for one sort (algorithmic bytes, not the
    traffic a kernel ends up causing):
      B_min = 8 (n+1) offsets + sum_i 8 ceil(max(d_i, 1) / 8) distinguishing
              prefix words + 8 n perm and LCP writes, with d_i = min(|s_i|,
              max(lcp_i, lcp_{i+1}) + 1) from the output;
      B_alg = B_min + 26 per string and distribution pass (idx u32, key u64,
              r u8 read and written).
    Re-gathers of equality buckets and base-case refinements are not
    counted, so B_alg is a lower bound."""
    import numpy as np
    n = len(perm)
    lens = np.diff(o.astype(np.int64))[perm.astype(np.int64)]
    L = lcp.astype(np.int64)
    nxt = np.append(L[1:], 0)
    d = np.minimum(lens, np.maximum(L, nxt) + 1)
    words = (np.maximum(d, 1) + 7) // 8
    b_min = 8 * (n + 1) + 8 * int(words.sum()) + 8 * n
    return b_min, b_min + 26 * int(dist_strings)


def copy_bandwidth(nbytes=2 << 30, reps=5):
    """Achievable HBM bandwidth: the library's streaming copy of `nbytes`,
    read + write bytes over the median event time."""
    import torch

    import paper_1808_00963_amd as ss
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    stream = torch.cuda.current_stream()
    ms = event_ms(lambda: ss.hbm_copy(dst, src, stream), reps, stream)
    ok = bool(torch.equal(dst[:: 1 << 20], src[:: 1 << 20]))
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes_each_way": nbytes, "ms": ms, "gbs": 2 * nbytes / (ms * 1e-3) / 1e9, "copied": ok}


def sort_measure(workload, steps, warmup, mode="levels", breakdown=True, timed_kernel=None, cpu=False,
                 alphabet="bytes"):
    """One named workload: generation, warm-up sorts, a breakdown pass with
    HIP events around every kernel launch (untimed), then the timed region
    of `steps` complete sorts with events (on the sort's stream) only around
    the launches of one kernel.  Returns timing, per-kernel breakdown,
    statistics and the host copy of the output."""
    import numpy as np
    import torch

    import gen
    import paper_1808_00963_amd as ss

    model, n, seed = gen.WORKLOADS[workload]
    t0 = time.perf_counter()
    c, o = gen.generate(model, n, seed)
    N = int(o[-1])
    log(f"generated {workload}: n={n} N={N} in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    chars = torch.from_numpy(c).to(dev)
    offs = torch.from_numpy(o.view(np.int64)).to(dev)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    lcp = torch.empty(n, dtype=torch.int32, device=dev)
    ctx = ss.Context(0)
    ctx.set_config(mode=mode, alphabet=alphabet)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        ctx.sort(chars, offs, perm, lcp, stream=stream)
    ctx.sync(stream)
    stats = ctx.stats()
    kt = {}
    if breakdown:
        ctx.set_profiling(True)
        ctx.reset_kernel_times()
        for _ in range(steps):
            ctx.sort(chars, offs, perm, lcp, stream=stream)
        torch.cuda.synchronize()
        ctx.set_profiling(False)
        kt = ctx.kernel_times()
    if timed_kernel:
        ctx.set_profiling(True, only=timed_kernel)
        ctx.reset_kernel_times()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.sort(chars, offs, perm, lcp, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.sync(stream)
    dk = None
    if timed_kernel:
        ctx.set_profiling(False)
        dk = ctx.kernel_times()[timed_kernel]
    sec = (t1 - t0) / steps
    ph, lh = perm.cpu().numpy().view(np.uint32), lcp.cpu().numpy().view(np.uint32)
    del chars, offs, perm, lcp, ctx
    torch.cuda.empty_cache()
    return {"workload": workload, "model": model, "seed": seed, "n": n, "N": N, "sec": sec, "stats": stats,
            "kt": kt, "timed_kernel": dk, "chars": c, "offsets": o, "perm": ph, "lcp": lh}


def cpu_baselines(c, o, label):
    """The oracle timed on the host: all cores (chunk sorts + pairwise
    merges, the threads this process may use) and one thread, on the whole
    workload.  Both results are checked against each other."""
    import numpy as np

    import oracle
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        cores = min(cores, int(os.environ["OMP_NUM_THREADS"]))
    N, n = int(o[-1]), len(o) - 1
    t0 = time.perf_counter()
    pm, lm = oracle.sort_mt(c, o, cores)
    dt_mt = time.perf_counter() - t0
    t0 = time.perf_counter()
    p1, l1 = oracle.sort(c, o)
    dt_1 = time.perf_counter() - t0
    same = bool(np.array_equal(pm, p1) and np.array_equal(lm, l1))
    log(f"oracle: {cores} threads {dt_mt:.2f} s, 1 thread {dt_1:.2f} s, identical {same}")
    mt = {"value": N / dt_mt, "unit": "chars/s", "cores": cores, "kind": "oracle",
          "sample": f"all {n} strings ({N} chars) of {label}, chunk qsort+memcmp sorts on {cores} threads, "
                    f"pairwise merges, brute LCP, {dt_mt:.2f} s", "strings_per_s": n / dt_mt}
    one = {"value": N / dt_1, "unit": "chars/s", "cores": 1, "kind": "oracle",
           "sample": f"all {n} strings of {label}, qsort+memcmp and brute LCP, 1 thread, {dt_1:.2f} s",
           "strings_per_s": n / dt_1, "identical_to_all_cores": same}
    return mt, one


def run_plain(args):
    """Default: the 16M-string Markov workload (the headline), plus the
    other workloads as extra keys unless --no-extras."""
    import numpy as np

    bpu = dict(BYTES_PER_UNIT)
    r = sort_measure(args.workload, args.steps, args.warmup, mode=args.sort_mode, timed_kernel="k_scatter",
                     alphabet=args.alphabet)
    n, N, sec, kt, stats = r["n"], r["N"], r["sec"], r["kt"], r["stats"]
    L = np.diff(r["offsets"].astype(np.int64))
    bpu["k_init"] = 8.0 + float(np.minimum(L, 8).mean()) + 13.0
    for k, v in sorted(kt.items(), key=lambda kv: -kv[1]["total_ms"]):
        if v["launches"]:
            per = v["total_ms"] / args.steps
            gbs = (v["units"] * bpu[k] / (v["total_ms"] * 1e-3) / 1e9) if k in bpu and v["total_ms"] else float("nan")
            log(f"{k:14s} {per:8.3f} ms/step  launches/step {v['launches'] / args.steps:6.1f}  "
                f"{v['units'] / args.steps:12.0f} {v['unit']}/step  {gbs:8.1f} GB/s alg")
    kernel_ms = sum(v["total_ms"] for v in kt.values()) / args.steps
    log(f"step {sec * 1e3:.3f} ms, kernels {kernel_ms:.3f} ms, stats {stats}")
    # roofline of the dominant kernel from the timed region's events
    dom = "k_scatter"
    d = r["timed_kernel"]
    avg_ms = d["total_ms"] / d["launches"]
    units_per_launch = d["units"] / d["launches"]
    alg_per_launch = units_per_launch * bpu[dom]
    achieved = alg_per_launch / (avg_ms * 1e-3) / 1e9
    impl_achieved = units_per_launch * SCATTER_IMPL_BYTES / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(dom, args.workload)
    # whole sort: the method's byte model and, when the committed counter
    # summary matches these kernels, the counted bytes
    dist_strings = kt.get("k_scatter", {}).get("units", 0.0) / max(1, args.steps)
    b_min, b_alg = alg_bytes(r["offsets"], r["perm"], r["lcp"], dist_strings)
    counted = measured_traffic("__sort__", args.workload)
    whole = {"b_min": b_min, "b_alg": b_alg, "alg_frac": b_alg / sec / (HBM_PEAK_GBS * 1e9),
             "counted_bytes": counted, "counted_frac": counted / sec / (HBM_PEAK_GBS * 1e9) if counted else None,
             "amplification": counted / b_alg if counted else None,
             "distribution_strings_per_sort": dist_strings}
    copy = copy_bandwidth()
    log(f"copy {copy['gbs']:.0f} GB/s; whole sort: B_alg {b_alg / 1e9:.3f} GB = {whole['alg_frac']:.3f} of peak")
    cpu = cpu1 = None
    if not args.no_cpu_baseline:
        cpu, cpu1 = cpu_baselines(r["chars"], r["offsets"], args.workload)
    out = {
        "metric": METRIC,
        "value": N / sec,
        "unit": "chars/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": args.workload, "model": r["model"], "seed": r["seed"], "n_strings": n, "n_chars": N,
                   "parallelism": "single-gpu", "mode": args.sort_mode, "alphabet": args.alphabet},
        "strings_per_s": n / sec,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": alg_per_launch, "bytes_per_string": bpu[dom],
                     "avg_launch_ms": avg_ms, "launches": d["launches"],
                     "frac_impl_bytes": impl_achieved / HBM_PEAK_GBS, "impl_bytes_per_string": SCATTER_IMPL_BYTES},
        "hbm_whole_sort": whole,
        "copy_calibration": copy,
        "cpu_baseline": cpu,
        "cpu_baseline_1thread": cpu1,
        "stats": stats,
        "kernel_ms_per_step": {k: v["total_ms"] / args.steps for k, v in kt.items() if v["launches"]},
    }
    del r
    if not args.no_extras:
        extras = {}
        for w in ("c2a_urls_8m", "c2b_suffixes_2m", "c0_random_128k"):
            e = sort_measure(w, args.steps, 2, mode=args.sort_mode, breakdown=True)
            top = sorted(((k, v["total_ms"] / args.steps) for k, v in e["kt"].items() if v["launches"]),
                         key=lambda kv: -kv[1])[:4]
            extras[w] = {"ms_per_sort": e["sec"] * 1e3, "chars_per_s": e["N"] / e["sec"],
                         "strings_per_s": e["n"] / e["sec"], "n_strings": e["n"], "n_chars": e["N"],
                         "levels": e["stats"]["levels"], "key_chars": e["stats"]["key_chars"],
                         "top_kernels_ms": dict(top)}
            log(f"{w}: {e['sec'] * 1e3:.3f} ms, {e['N'] / e['sec'] / 1e9:.1f} G chars/s, levels "
                f"{e['stats']['levels']}, {e['stats']['key_chars']} chars per key, top {top}")
            del e
            if w == "c2b_suffixes_2m":  # DNA: the same workload with alphabet-compressed keys
                e = sort_measure(w, args.steps, 2, mode=args.sort_mode, breakdown=False, alphabet="compress")
                extras[w]["ms_per_sort_compressed_keys"] = e["sec"] * 1e3
                extras[w]["compressed_key_chars"] = e["stats"]["key_chars"]
                log(f"{w} with compressed keys ({e['stats']['key_chars']} per key): {e['sec'] * 1e3:.3f} ms")
                del e
        extras["batched_4096_sets"] = batch_measure(max(4, args.steps // 2))
        extras["serving"] = serve_measure(args.pool, args.requests, args.serve_warmup)
        out["extras"] = extras
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
