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
#   k_init      per string: offset (8) + first word (<= 8, measured) + element write (16)
#   k_classify  per string: element read (16) + bucket id write (2)
#   k_scatter   per string: bucket id (2) + element read (16) + element write (16)
#   k_base      per string: element read (16) + perm and lcp writes (4 + 4)
#   k_scan      per counter: reduce read (4) + scan read (4) + write (4)
#   k_lcp_fill  per boundary: entry (8) + lcp (4+4) + perm (8) + offsets (32) + two words (16)
BYTES_PER_UNIT = {
    "k_classify": 18.0,
    "k_scatter": 34.0,
    "k_base": 24.0,
    "k_base_wave1": 24.0,
    "k_base_wave2": 24.0,
    "k_base_wave4": 24.0,
    "k_scan": 12.0,
    "k_lcp_fill": 72.0,
}


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


def run_batch(args):
    """Batched workload: 4096 independent sets (character budgets
    log-uniform in [1e3, 1e6], model per set uniform over the four
    generators).  Compares a loop of per-set ss_sort calls on one stream with
    the batched forms (host-driven levels, one persistent launch, hipGraph of
    the persistent launch).  All forms must give identical outputs."""
    import ctypes

    import numpy as np
    import torch

    import gen
    import paper_1808_00963_amd as ss

    t0 = time.perf_counter()
    c, o, sb = gen.batch_sets(num_sets=args.sets)
    n, N, S = len(o) - 1, int(o[-1]), len(sb) - 1
    print(f"[bench] batched workload: {S} sets, n={n} N={N} ({time.perf_counter() - t0:.1f}s)", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    chars = torch.from_numpy(c).to(dev)
    offs = torch.from_numpy(o.view(np.int64)).to(dev)
    sbd = torch.from_numpy(sb.astype(np.int32)).to(dev)
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    ctx = ss.Context(0)
    lib = ss.lib()
    outs = {}

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            a = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - a)
        return float(np.median(ts))

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

    results = {}
    ctx.set_config(mode="levels")
    results["per_set_launches"] = timed(per_set, max(1, args.steps // 4))
    outs["per_set_launches"] = (perm.clone(), lcp.clone())
    results["batched_levels"] = timed(lambda: ctx.sort_batch(chars, offs, sbd, perm, lcp, stream), args.steps)
    outs["batched_levels"] = (perm.clone(), lcp.clone())
    ctx.set_config(mode="host_levels")
    results["batched_host_levels"] = timed(lambda: ctx.sort_batch(chars, offs, sbd, perm, lcp, stream), args.steps)
    outs["batched_host_levels"] = (perm.clone(), lcp.clone())
    ctx.set_config(mode="persistent")
    results["batched_persistent"] = timed(lambda: ctx.sort_batch(chars, offs, sbd, perm, lcp, stream), args.steps)
    outs["batched_persistent"] = (perm.clone(), lcp.clone())
    ctx.set_config(mode="levels")
    g = ctx.graph_batch(chars, offs, sbd, perm, lcp)

    def graph_run():
        g.launch(stream)
        ctx.sync(stream)

    results["batched_graph"] = timed(graph_run, args.steps)
    outs["batched_graph"] = (perm.clone(), lcp.clone())
    g.close()
    # autotuned batched form: the tuner times its grid on this batch, then
    # the chosen configuration is timed like the others
    tctx = ss.Context(0)
    t_a = time.perf_counter()
    tuned_cfg, tuned_ms, _, _ = tctx.autotune(chars, offs, sbd, perm, lcp, reps=2, stream=stream)
    tune_s = time.perf_counter() - t_a
    results["batched_autotuned"] = timed(lambda: tctx.sort_batch(chars, offs, sbd, perm, lcp, stream), args.steps)
    outs["batched_autotuned"] = (perm.clone(), lcp.clone())
    ref = outs["per_set_launches"]
    identical = all(torch.equal(v[0], ref[0]) and torch.equal(v[1], ref[1]) for v in outs.values())
    for k, v in results.items():
        print(f"[bench] {k:22s} {v * 1e3:9.2f} ms  {N / v / 1e9:8.2f} G chars/s", file=sys.stderr, flush=True)
    best = min(("batched_levels", "batched_host_levels", "batched_persistent", "batched_graph", "batched_autotuned"),
               key=lambda k: results[k])
    out = {
        "metric": METRIC,
        "value": N / results[best],
        "unit": "chars/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": results[best] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "batched_4096_sets", "sets": S, "n_strings": n, "n_chars": N, "form": best},
        "batched_vs_per_set": results["per_set_launches"] / results[best],
        "ms": {k: v * 1e3 for k, v in results.items()},
        "outputs_identical": identical,
        "autotune": {"config": tuned_cfg, "tuner_median_ms": tuned_ms, "tuning_s": tune_s},
    }
    print(json.dumps(out), flush=True)


def run_serve(args):
    """Serving workload: a Poisson stream of sort requests, sizes log-uniform
    in [1e3, 1e6] strings from the Markov generator, admitted by an 8 GB HBM
    budget.  Saturation throughput mu is measured closed-loop first; the
    open-loop runs at 0.5 mu and 0.8 mu report p50/p99 latency (submit ->
    outputs on the host) and chars/s.  Requests cycle through a pool of
    distinct pre-generated requests held in pinned host memory."""
    import threading

    import numpy as np
    import torch

    import gen
    import paper_1808_00963_amd as ss

    seed, P = 6, args.pool
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
    chars_of = np.array([int(o[-1]) for _, o in pool])
    print(f"[bench] serving pool: {P} requests, mean {sizes.mean():.0f} strings / {chars_of.mean() / 1e6:.2f} MB "
          f"({time.perf_counter() - t0:.1f}s)", file=sys.stderr, flush=True)
    srv = ss.Server(8 << 30, max_inflight=4096)

    # closed loop: keep the queue full, measure completions per second
    for j in range(min(P, 32)):
        srv.wait(srv.submit(*pool[j]))
    srv.reset_stats()
    K = args.requests
    a = time.perf_counter()
    tickets = [srv.submit(*pool[j % P]) for j in range(min(K, 600))]
    for t in tickets:
        srv.wait(t)
    dt = time.perf_counter() - a
    mu = len(tickets) / dt
    sat = srv.stats()
    print(f"[bench] saturation: {mu:.1f} req/s, {sat['chars_completed'] / dt / 1e9:.2f} G chars/s, "
          f"inflight_max {sat['inflight_max']}", file=sys.stderr, flush=True)

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
                tickets[j] = (srv.submit(*pool[j % P]), time.perf_counter())

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
        return {"rate_req_s": rate, "requests": n_req - warm, "p50_ms": float(np.percentile(L, 50)),
                "p99_ms": float(np.percentile(L, 99)), "mean_ms": float(L.mean()),
                "chars_per_s": done_chars / (t_end - t_first), "inflight_max": st["inflight_max"],
                "footprint_max_gb": st["footprint_max"] / 1e9}

    res = {}
    for frac in (0.5, 0.8):
        r = open_loop(frac * mu, K + args.serve_warmup, args.serve_warmup)
        res[str(frac)] = r
        print(f"[bench] rate {frac:.1f} mu = {r['rate_req_s']:.1f} req/s: p50 {r['p50_ms']:.2f} ms, p99 "
              f"{r['p99_ms']:.2f} ms, {r['chars_per_s'] / 1e9:.2f} G chars/s, inflight_max {r['inflight_max']}",
              file=sys.stderr, flush=True)
    srv.close()
    main_r = res["0.8"]
    out = {
        "metric": METRIC,
        "value": main_r["chars_per_s"],
        "unit": "chars/s",
        "n_gpus": 1,
        "steps": main_r["requests"],
        "warmup": args.serve_warmup,
        "ms_per_step": main_r["mean_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "serving_poisson_markov", "budget_bytes": 8 << 30, "pool": P,
                   "sizes": "log-uniform 1e3..1e6 strings", "rate": "0.8 x saturation"},
        "saturation_req_s": mu,
        "p50_ms": main_r["p50_ms"],
        "p99_ms": main_r["p99_ms"],
        "open_loop": res,
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
    for _ in range(args.warmup + args.steps):
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
        base = name.split("(")[0].replace("void ", "").replace("ss::", "")
        return {"k_base_wave<1>": "k_base_wave1", "k_base_wave<2>": "k_base_wave2",
                "k_base_wave<4>": "k_base_wave4"}.get(base, base)

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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--mode", choices=["plain", "batch", "serve", "profile", "traffic", "merge", "sa"], default="plain")
    ap.add_argument("--fetch-csv", help="traffic mode: rocprofv3 counter_collection.csv of the FETCH_SIZE run")
    ap.add_argument("--write-csv", help="traffic mode: rocprofv3 counter_collection.csv of the WRITE_SIZE run")
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
    ap.add_argument("--sort-mode", default="levels", choices=["levels", "host_levels", "persistent"],
                    help="how the recursion levels are driven (ss_config.mode)")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="strings for the oracle timing (a prefix of the workload; 0 = all)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on exactly one GPU (asked for {args.gpus}); "
              "the sort is single-GPU and multi-GPU sharding is not implemented.", file=sys.stderr)
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
    if args.mode == "merge":
        run_merge(args)
        return
    if args.mode == "sa":
        run_sa(args)
        return

    import numpy as np
    import torch

    import gen
    import paper_1808_00963_amd as ss

    model, n, seed = gen.WORKLOADS[args.workload]
    t0 = time.perf_counter()
    c, o = gen.generate(model, n, seed)
    N = int(o[-1])
    print(f"[bench] generated {args.workload}: n={n} N={N} in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    chars = torch.from_numpy(c).to(dev)
    offs = torch.from_numpy(o.view(np.int64)).to(dev)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    lcp = torch.empty(n, dtype=torch.int32, device=dev)
    ctx = ss.Context(0)
    ctx.set_config(mode=args.sort_mode)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        ctx.sort(chars, offs, perm, lcp, stream=stream)
    torch.cuda.synchronize()
    stats = ctx.stats()

    # breakdown pass (untimed): HIP events around every kernel launch
    ctx.set_profiling(True)
    ctx.reset_kernel_times()
    for _ in range(args.steps):
        ctx.sort(chars, offs, perm, lcp, stream=stream)
    torch.cuda.synchronize()
    ctx.set_profiling(False)
    kt = ctx.kernel_times()
    bpu = dict(BYTES_PER_UNIT)
    L = np.diff(o)
    bpu["k_init"] = 8.0 + float(np.minimum(L, 8).mean()) + 16.0
    dom = max((k for k in kt if k in bpu and kt[k]["launches"]), key=lambda k: kt[k]["total_ms"])

    # timed region: K complete sorts; HIP events (on the sort's stream) only
    # around the launches of the dominant kernel
    ctx.set_profiling(True, only=dom)
    ctx.reset_kernel_times()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.sort(chars, offs, perm, lcp, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.set_profiling(False)
    d = ctx.kernel_times()[dom]

    sec = (t1 - t0) / args.steps
    value = N / sec
    strings_per_s = n / sec

    # roofline of the dominant kernel, from the timed region's events
    alg_bytes_per_launch = d["units"] / d["launches"] * bpu[dom]
    avg_ms = d["total_ms"] / d["launches"]
    achieved = alg_bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(dom, args.workload)
    for k, v in sorted(kt.items(), key=lambda kv: -kv[1]["total_ms"]):
        if v["launches"]:
            per = v["total_ms"] / args.steps
            gbs = (v["units"] * bpu[k] / (v["total_ms"] * 1e-3) / 1e9) if k in bpu and v["total_ms"] else float("nan")
            print(f"[bench] {k:12s} {per:8.3f} ms/step  launches/step {v['launches'] / args.steps:6.1f}  "
                  f"{v['units'] / args.steps:12.0f} {v['unit']}/step  {gbs:8.1f} GB/s alg", file=sys.stderr)
    kernel_ms = sum(v["total_ms"] for v in kt.values()) / args.steps
    print(f"[bench] step {sec * 1e3:.3f} ms, kernels {kernel_ms:.3f} ms, stats {stats}", file=sys.stderr, flush=True)

    # CPU baseline: the oracle as it is, single thread, on the host cores
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        ns = n if args.cpu_sample <= 0 else min(n, args.cpu_sample)
        oc = c[: int(o[ns])]
        oo = o[: ns + 1]
        t0 = time.perf_counter()
        oracle.sort(oc, oo)
        dt = time.perf_counter() - t0
        cpu = {"value": int(oo[-1]) / dt, "unit": "chars/s", "cores": 1, "kind": "oracle",
               "sample": f"first {ns} strings ({int(oo[-1])} chars) of {args.workload}, qsort+memcmp and brute LCP, "
                         f"1 thread, {dt:.2f} s"}
        print(f"[bench] oracle {dt:.2f}s on {ns} strings", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": value,
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
        "config": {"workload": args.workload, "model": model, "seed": seed, "n_strings": n, "n_chars": N,
                   "parallelism": "single-gpu"},
        "strings_per_s": strings_per_s,
        "hbm_frac_alg_whole_sort": None,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": alg_bytes_per_launch, "avg_launch_ms": avg_ms},
        "cpu_baseline": cpu,
        "kernel_ms_per_step": {k: v["total_ms"] / args.steps for k, v in kt.items() if v["launches"]},
    }
    # whole-sort algorithmic bytes over the step time
    alg_total = sum(v["units"] * bpu[k] for k, v in kt.items() if k in bpu) / args.steps
    out["hbm_frac_alg_whole_sort"] = alg_total / sec / (HBM_PEAK_GBS * 1e9)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
