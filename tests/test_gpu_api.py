"""Library services on the GPU: statistics, per-kernel timing (all kernels or
one), the streaming copy, explicit output buffers and streams."""
import sys

import numpy as np
import pytest
import torch

import gen
from gpu_util import assert_equal_to_oracle, needs_gpu, to_device, to_host

pytestmark = [pytest.mark.gpu, needs_gpu]


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_stats_account_for_every_string():
    """Every string ends in exactly one place: a base case, a singleton bucket
    or an identical-string bucket; the per-class base-case counts add up and
    the class bounds hold."""
    import paper_1808_00963_amd as ss
    note("case stats")
    c, o = gen.generate("markov", 200000, 3)
    cd, od = to_device(c, o)
    ctx = ss.Context()
    p, l = ctx.sort(cd, od)
    torch.cuda.synchronize()
    assert_equal_to_oracle(c, o, to_host(p), to_host(l), full=False)
    st = ctx.stats()
    assert st["levels"] >= 2
    assert sum(st["base_segments_by_class"]) == st["base_segments"]
    assert sum(st["base_strings_by_class"]) <= len(o) - 1
    bounds = [64, 128, 256, 1024]
    for q, (segs, strs) in enumerate(zip(st["base_segments_by_class"], st["base_strings_by_class"])):
        assert strs <= segs * bounds[q]
        if q and segs:
            assert strs > segs * bounds[q - 1]
    assert st["pending_lcps"] >= st["base_segments"] - st["dist_segments"]


def test_profiling_all_and_only_one_kernel():
    import paper_1808_00963_amd as ss
    note("case profiling")
    c, o = gen.generate("markov", 300000, 4)
    cd, od = to_device(c, o)
    ctx = ss.Context()
    ctx.sort(cd, od)
    ctx.set_profiling(True)
    ctx.reset_kernel_times()
    ctx.sort(cd, od)
    torch.cuda.synchronize()
    kt = ctx.kernel_times()
    assert kt["k_init"]["launches"] == 1 and kt["k_init"]["units"] == len(o) - 1
    assert kt["k_scatter"]["launches"] >= 1 and kt["k_scatter"]["total_ms"] > 0
    assert kt["k_classify"]["units"] == kt["k_scatter"]["units"]
    ctx.set_profiling(True, only="k_scatter")
    ctx.reset_kernel_times()
    ctx.sort(cd, od)
    torch.cuda.synchronize()
    kt1 = ctx.kernel_times()
    assert kt1["k_scatter"]["launches"] == kt["k_scatter"]["launches"]
    assert all(v["launches"] == 0 for k, v in kt1.items() if k != "k_scatter")
    with pytest.raises(ss.SSError):
        ctx.set_profiling(True, only="no_such_kernel")
    ctx.set_profiling(False)


def test_hbm_copy_moves_bytes_exactly():
    import paper_1808_00963_amd as ss
    note("case hbm copy")
    src = torch.randint(0, 256, (3 << 20,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    ss.hbm_copy(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    with pytest.raises(ValueError):
        ss.hbm_copy(dst[:16], src)


def test_caller_buffers_and_side_stream():
    """Outputs written into caller-owned buffers on a caller's stream; the
    result is ready after that stream is synchronised."""
    import paper_1808_00963_amd as ss
    note("case side stream")
    c, o = gen.generate("urls", 50000, 6)
    cd, od = to_device(c, o)
    n = len(o) - 1
    perm = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    lcp = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    ctx = ss.Context()
    with torch.cuda.stream(s):
        ctx.sort(cd, od, perm, lcp, stream=s)
    s.synchronize()
    assert_equal_to_oracle(c, o, to_host(perm), to_host(lcp))


def test_sorts_are_stream_ordered_and_asynchronous():
    """The sort call only enqueues: work enqueued after it on the same stream
    (here a copy of the outputs) sees the finished outputs, and two sorts of
    one context issued on different streams run one after the other (they
    share the context's workspace); everything is checked only after the
    device is synchronised."""
    import paper_1808_00963_amd as ss
    note("case async ordering")
    c1, o1 = gen.generate("markov", 300000, 8)
    c2, o2 = gen.generate("urls", 200000, 9)
    d1, d2 = to_device(c1, o1), to_device(c2, o2)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ctx = ss.Context()
    with torch.cuda.stream(s1):
        p1, l1 = ctx.sort(*d1, stream=s1)
        p1c, l1c = p1.clone(), l1.clone()
    with torch.cuda.stream(s2):
        p2, l2 = ctx.sort(*d2, stream=s2)
        p2c, l2c = p2.clone(), l2.clone()
    torch.cuda.synchronize()
    ctx.sync()
    assert_equal_to_oracle(c1, o1, to_host(p1c), to_host(l1c), label="stream 1")
    assert_equal_to_oracle(c2, o2, to_host(p2c), to_host(l2c), label="stream 2")


def test_level_budget_and_persistent_tail():
    """A fresh context enqueues a few level launches; a sort that needs more
    levels finishes them in the persistent tail, and the next sort on the
    context enqueues as many level launches as the last one needed.  Both
    results equal the oracle."""
    import paper_1808_00963_amd as ss
    note("case level budget")
    n, L = 30000, 150
    rng = np.random.default_rng(12)
    rows = rng.integers(ord("a"), ord("d"), (n, L), dtype=np.uint8)
    rows[:, :100] = ord("k")  # a shared prefix: one equality bucket per 8 characters
    # a few strings leave the prefix at the start of every word, so no level
    # can skip more than the one word of its equality bucket
    for j in range(1, 13):
        rows[40 * j:40 * j + 40, 8 * j] = ord("a")
    c = rows.reshape(-1)
    o = np.arange(n + 1, dtype=np.uint64) * L
    cd, od = to_device(c, o)
    ctx = ss.Context()
    ctx.set_config(alphabet="bytes")  # 8 characters per level: more than 10 levels
    for rep in range(2):
        p, l = ctx.sort(cd, od)
        torch.cuda.synchronize()
        assert_equal_to_oracle(c, o, to_host(p), to_host(l), label=f"rep {rep}")
        assert ctx.stats()["levels"] > 10


def shared_prefix_cases():
    """Inputs whose large equality buckets share long prefixes."""
    rng = np.random.default_rng(31)
    out = []
    # one prefix of 100 characters shared by all strings
    n, L = 30000, 150
    rows = rng.integers(ord("a"), ord("d"), (n, L), dtype=np.uint8)
    rows[:, :100] = ord("k")
    out.append(("prefix 100", rows.reshape(-1), np.arange(n + 1, dtype=np.uint64) * L))
    # a prefix longer than one step can skip
    n, L = 12000, 760
    rows = rng.integers(ord("a"), ord("e"), (n, L), dtype=np.uint8)
    rows[:, :700] = rng.integers(ord("a"), ord("z"), 700, dtype=np.uint8)
    out.append(("prefix 700", rows.reshape(-1), np.arange(n + 1, dtype=np.uint64) * L))
    # groups with prefixes of their own lengths behind a common one, plus
    # exact duplicates of a few long strings and strings ending inside the
    # prefixes
    strings = []
    for g in range(24):
        plen = int(rng.integers(20, 220))
        pre = bytes(rng.integers(ord("a"), ord("z"), plen, dtype=np.uint8))
        for _ in range(int(rng.integers(1100, 2600))):
            tail = bytes(rng.integers(ord("a"), ord("c"), int(rng.integers(0, 12)), dtype=np.uint8))
            strings.append(b"http://www.site" + pre + tail)
    for _ in range(3):
        s = bytes(rng.integers(ord("a"), ord("z"), 300, dtype=np.uint8))
        strings += [s] * 3000
    for _ in range(2000):
        s = strings[int(rng.integers(0, len(strings)))]
        strings.append(s[:int(rng.integers(0, len(s) + 1))])
    order = rng.permutation(len(strings))
    strings = [strings[i] for i in order]
    c, o = gen.from_list(strings)
    out.append(("groups", c, o))
    return out


@pytest.mark.parametrize("mode", ["levels", "host_levels", "persistent"])
def test_equality_buckets_skip_shared_prefixes(mode):
    """Large equality buckets whose members all share the word after the
    splitter's skip that word too (checked in the scatter of the level
    modes; the persistent mode advances one word): every mode equals the
    oracle, and the 100-character prefix takes fewer levels than one per
    word."""
    import paper_1808_00963_amd as ss
    for label, c, o in shared_prefix_cases():
        note(f"case shared prefix {label} mode {mode}")
        cd, od = to_device(c, o)
        ctx = ss.Context()
        ctx.set_config(mode=mode, alphabet="bytes")
        for rep in range(2):  # the second sort reuses the workspace and its tree arrays
            p, l = ctx.sort(cd, od)
            torch.cuda.synchronize()
            assert_equal_to_oracle(c, o, to_host(p), to_host(l), label=f"{label} {mode} rep {rep}")
        if label == "prefix 100" and mode != "persistent":
            assert ctx.stats()["levels"] <= 9  # one word per level would take more than 12


def test_shared_prefixes_with_compressed_keys():
    """A shared prefix with keys of 2 bits per character (32 characters per
    word): the skipped word is a compressed word."""
    import paper_1808_00963_amd as ss
    rng = np.random.default_rng(32)
    n, L = 20000, 400
    rows = rng.integers(ord("a"), ord("d"), (n, L), dtype=np.uint8)
    rows[:, :300] = rng.integers(ord("a"), ord("d"), 300, dtype=np.uint8)
    rows[:500, 150] = (rows[0, 150] - ord("a") + 1) % 3 + ord("a")  # a few leave the prefix in the middle
    c = rows.reshape(-1)
    o = np.arange(n + 1, dtype=np.uint64) * L
    note("case shared prefix compressed")
    cd, od = to_device(c, o)
    ctx = ss.Context()
    ctx.set_config(alphabet="compress")
    p, l = ctx.sort(cd, od)
    torch.cuda.synchronize()
    assert_equal_to_oracle(c, o, to_host(p), to_host(l), label="compressed")
    assert ctx.stats()["key_chars"] == 32
