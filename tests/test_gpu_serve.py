"""Serving form on the GPU: continuous batching under an HBM budget.

Each request's result must be the same alone and in the mix (bit-exact, equal
to the oracle), admission must never exceed the budget, and requests that
arrive while others run must share the device with them."""
import sys
import threading
import time

import numpy as np
import pytest

import gen
import oracle
from gpu_util import needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def request_pool(k, seed=40, lo=1e3, hi=2e5):
    """k requests from the Markov generator, sizes log-uniform in [lo, hi]."""
    out = []
    for j in range(k):
        n = gen.log_uniform(seed, j, lo, hi)
        out.append(gen.generate("markov", n, gen.mix(seed, j)))
    return out


def expect(req):
    return oracle.sort(*req)


def test_alone_and_in_the_mix_are_identical():
    import paper_1808_00963_amd as ss
    note("case serve alone vs mix")
    reqs = request_pool(24)
    reqs += [gen.generate(m, 3000, 9) for m in ("urls", "suffixes", "bytes", "binary")]
    reqs += [gen.from_list([]), gen.from_list([b"only"]), gen.from_list([b"b", b"a", b"b", b""])]
    exp = [expect(r) for r in reqs]
    srv = ss.Server(2 << 30, max_inflight=64)
    # alone: one request at a time
    alone = []
    for r in reqs:
        t = srv.submit(*r)
        alone.append(srv.wait(t)[:2])
    # in the mix: all at once, from two threads
    tickets = [None] * len(reqs)

    def submit(idx):
        for i in idx:
            tickets[i] = srv.submit(*reqs[i])
    th = [threading.Thread(target=submit, args=(range(k, len(reqs), 2),)) for k in (0, 1)]
    [t.start() for t in th]
    [t.join() for t in th]
    mix = [srv.wait(t)[:2] for t in tickets]
    st = srv.stats()
    srv.close()
    for i, (a, m, e) in enumerate(zip(alone, mix, exp)):
        assert np.array_equal(a[0], e[0]) and np.array_equal(a[1], e[1]), f"alone {i}"
        assert np.array_equal(m[0], e[0]) and np.array_equal(m[1], e[1]), f"mix {i}"
    assert st["inflight_max"] >= 2
    assert st["completed"] == 2 * len(reqs)


def test_requests_join_a_running_batch():
    """A large request is running; small ones submitted meanwhile finish
    before it (they join its levels instead of waiting behind it)."""
    import paper_1808_00963_amd as ss
    note("case serve join")
    big = gen.generate("suffixes", 400000, 4)
    small = request_pool(8, seed=41, lo=1e3, hi=5e3)
    srv = ss.Server(4 << 30, max_inflight=64)
    tb = srv.submit(*big)
    time.sleep(0.002)
    ts = [srv.submit(*r) for r in small]
    done_small = [srv.wait(t) for t in ts]
    res_big = srv.wait(tb)
    st = srv.stats()
    srv.close()
    for r, (p, l, _) in zip(small, done_small):
        e = expect(r)
        assert np.array_equal(p, e[0]) and np.array_equal(l, e[1])
    code = oracle.check(*big, res_big[0], res_big[1])
    assert code == -1, oracle.describe_check(code, len(res_big[0]))
    assert st["inflight_max"] >= 2


def test_budget_is_respected_and_queue_drains():
    import paper_1808_00963_amd as ss
    note("case serve budget")
    budget = 96 << 20
    srv = ss.Server(budget, max_inflight=16)
    reqs = request_pool(20, seed=42, lo=2e4, hi=1.5e5)
    fps = [srv.footprint(len(o) - 1, int(o[-1])) for _, o in reqs]
    ts = [srv.submit(*r) for r in reqs]
    res = [srv.wait(t) for t in ts]
    st = srv.stats()
    for r, (p, l, _) in zip(reqs, res):
        e = expect(r)
        assert np.array_equal(p, e[0]) and np.array_equal(l, e[1])
    assert st["footprint_max"] <= st["arena_bytes"] <= budget
    assert sum(fps) > st["arena_bytes"]          # the requests could not all fit at once
    # a request larger than the whole arena is rejected, the server keeps working
    too_big = gen.generate("markov", 2000000, 7)
    with pytest.raises(ss.SSError) as e:
        srv.submit(*too_big)
    assert e.value.status == ss.SS_REJECTED
    r = reqs[0]
    p, l, _ = srv.wait(srv.submit(*r))
    assert np.array_equal(p, expect(r)[0])
    srv.close()


def test_malformed_request_is_rejected_and_others_unaffected():
    import paper_1808_00963_amd as ss
    note("case serve malformed")
    srv = ss.Server(1 << 30, max_inflight=8)
    good = request_pool(3, seed=43)
    c, o = gen.generate("random", 500, 1)
    bad = o.copy()
    bad[10], bad[11] = bad[11], bad[10]
    t0 = srv.submit(*good[0])
    with pytest.raises(ss.SSError) as e:
        srv.submit(c, bad)
    assert e.value.status == ss.SS_LIMIT
    ts = [t0] + [srv.submit(*g) for g in good[1:]]
    for g, t in zip(good, ts):
        p, l, _ = srv.wait(t)
        assert np.array_equal(p, expect(g)[0]) and np.array_equal(l, expect(g)[1])
    srv.close()


def test_cancel_queued_request():
    import paper_1808_00963_amd as ss
    note("case serve cancel")
    srv = ss.Server(64 << 20, max_inflight=2)
    reqs = request_pool(6, seed=44, lo=1e5, hi=1.5e5)
    ts = [srv.submit(*r) for r in reqs]
    cancelled = None
    for t in reversed(ts):        # the last ones are still queued
        try:
            srv.cancel(t)
            cancelled = t
            break
        except ss.SSError:
            pass
    for r, t in zip(reqs, ts):
        if t == cancelled:
            continue
        p, l, _ = srv.wait(t)
        assert np.array_equal(p, expect(r)[0])
    st = srv.stats()
    assert st["cancelled"] == (1 if cancelled else 0)
    srv.close()


def test_serving_workload_sizes_8gb_budget():
    """Requests of the serving workload's sizes: Markov requests of 2e5 to
    1e6 strings (the upper part of its log-uniform range) under its 8 GB
    budget, submitted at once from three threads so that several are on the
    device together, then again one at a time; every result equals the
    oracle's check of that request, alone and in the mix identically, and
    the admitted footprint never exceeds the budget."""
    import paper_1808_00963_amd as ss
    note("case serve workload sizes")
    reqs = request_pool(10, seed=61, lo=2e5, hi=1e6)
    reqs.append(gen.generate("markov", 1000000, gen.mix(61, 99)))  # the largest size exactly
    srv = ss.Server(8 << 30, max_inflight=64)
    tickets = [None] * len(reqs)

    def submit(idx):
        for i in idx:
            tickets[i] = srv.submit(*reqs[i])
    th = [threading.Thread(target=submit, args=(range(k, len(reqs), 3),)) for k in (0, 1, 2)]
    [t.start() for t in th]
    [t.join() for t in th]
    mix = [srv.wait(t)[:2] for t in tickets]
    st = srv.stats()
    assert st["footprint_max"] <= 8 << 30
    assert st["inflight_max"] >= 2
    for i, (r, (p, l)) in enumerate(zip(reqs, mix)):
        n = len(r[1]) - 1
        assert 2e5 <= n <= 1e6
        code = oracle.check(r[0], r[1], p, l)
        assert code == -1, f"request {i} (n={n}) in the mix: {oracle.describe_check(code, n)}"
    for i, r in enumerate(reqs[:4]):
        p, l, _ = srv.wait(srv.submit(*r))
        assert np.array_equal(p, mix[i][0]) and np.array_equal(l, mix[i][1]), f"request {i} alone vs mix"
    srv.close()


def test_requests_with_shared_prefixes():
    """Requests whose large equality buckets skip shared words, submitted
    together with ordinary ones: each result equals the oracle's."""
    import paper_1808_00963_amd as ss
    note("case serve shared prefixes")
    rng = np.random.default_rng(44)
    reqs = request_pool(6, seed=45, hi=5e4)
    for j in range(4):
        pre = bytes(rng.integers(ord("a"), ord("z"), int(rng.integers(30, 150)), dtype=np.uint8))
        strings = [pre + bytes(rng.integers(ord("a"), ord("d"), int(rng.integers(0, 12)), dtype=np.uint8))
                   for _ in range(int(rng.integers(2000, 8000)))]
        reqs.append(gen.from_list(strings))
    reqs.append(gen.from_list([b"z" * 70] * 2500))  # exact duplicates
    exp = [expect(r) for r in reqs]
    srv = ss.Server(2 << 30, max_inflight=64)
    tickets = [srv.submit(*r) for r in reqs]
    got = [srv.wait(t)[:2] for t in tickets]
    srv.close()
    for i, (g, e) in enumerate(zip(got, exp)):
        assert np.array_equal(g[0], e[0]) and np.array_equal(g[1], e[1]), f"request {i}"
