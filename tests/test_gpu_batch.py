"""Batched form in every mode (device-driven levels, one persistent launch,
host-driven levels) and its hipGraph on the GPU: every set's result equals
the oracle's result for that set alone."""
import sys

import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import assert_equal_to_oracle, gpu_sort, needs_gpu, to_device, to_host

pytestmark = [pytest.mark.gpu, needs_gpu]


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def check_sets(c, o, sb, p, l, full=True):
    """Each set's slice of (perm, lcp) against the oracle on that set."""
    for j in range(len(sb) - 1):
        b, e = int(sb[j]), int(sb[j + 1])
        if e == b:
            continue
        cj = c[int(o[b]):int(o[e])]
        oj = o[b:e + 1] - o[b]
        assert_equal_to_oracle(cj, oj, p[b:e], l[b:e], full=full, label=f"set {j}")


def run_batch(c, o, sb, ctx=None):
    import paper_1808_00963_amd as ss
    ctx = ctx or ss.Context()
    cd, od = to_device(c, o)
    sbd = torch.from_numpy(sb.astype(np.int32)).cuda()
    p, l = ctx.sort_batch(cd, od, sbd)
    torch.cuda.synchronize()
    return to_host(p), to_host(l)


def small_batch(num_sets=64, seed=11, scale=0.02):
    return gen.batch_sets(num_sets=num_sets, seed=seed, scale=scale)


MODES = ["levels", "persistent", "host_levels"]


@pytest.mark.parametrize("mode", MODES)
def test_batch_vs_oracle(mode):
    import paper_1808_00963_amd as ss
    note(f"case batch mode={mode}")
    c, o, sb = small_batch()
    ctx = ss.Context()
    ctx.set_config(mode=mode)
    p, l = run_batch(c, o, sb, ctx)
    check_sets(c, o, sb, p, l)


@pytest.mark.parametrize("mode", MODES)
def test_batch_edge_sets(mode):
    import paper_1808_00963_amd as ss
    note(f"case batch edges mode={mode}")
    sets = [[], [b"x"], [b"b", b"a"], [b""] * 5, [b"ab", b"ab", b"a"], [bytes([255, 0])] * 3 + [b""],
            [b"q" * k for k in range(300)]]
    strings, sb = [], [0]
    for s in sets:
        strings += s
        sb.append(len(strings))
    c, o = gen.from_list(strings)
    sb = np.array(sb, dtype=np.uint32)
    ctx = ss.Context()
    ctx.set_config(mode=mode)
    p, l = run_batch(c, o, sb, ctx)
    check_sets(c, o, sb, p, l)


@pytest.mark.parametrize("model", ["random", "markov", "urls", "suffixes", "bytes", "binary"])
@pytest.mark.parametrize("n", [1, 2, 1000, 50000])
def test_persistent_single_vs_oracle(model, n):
    import paper_1808_00963_amd as ss
    note(f"case persistent model={model} n={n}")
    ctx = ss.Context()
    ctx.set_config(mode="persistent")
    c, o = gen.generate(model, n, 500 + n)
    p, l = gpu_sort(c, o, ctx=ctx)
    assert_equal_to_oracle(c, o, p, l, label=f"persistent {model}/{n}")


def test_persistent_full_size_markov():
    import paper_1808_00963_amd as ss
    note("case persistent full c1")
    ctx = ss.Context()
    ctx.set_config(mode="persistent")
    c, o = gen.workload("c1_markov_16m")
    p, l = gpu_sort(c, o, ctx=ctx)
    assert_equal_to_oracle(c, o, p, l, full=False, label="persistent c1")


def test_graph_replays_match_eager():
    import paper_1808_00963_amd as ss
    note("case graph replays")
    c, o, sb = small_batch(num_sets=48, seed=21)
    ctx = ss.Context()
    eager = run_batch(c, o, sb, ctx)
    check_sets(c, o, sb, *eager)
    cd, od = to_device(c, o)
    sbd = torch.from_numpy(sb.astype(np.int32)).cuda()
    n = len(o) - 1
    perm = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    lcp = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    g = ctx.graph_batch(cd, od, sbd, perm, lcp)
    assert g.levels >= 1
    stream = torch.cuda.current_stream()
    for rep in range(3):
        perm.fill_(-1)
        lcp.fill_(-1)
        g.launch(stream)
        ctx.sync(stream)
        assert np.array_equal(to_host(perm), eager[0]), f"replay {rep} perm"
        assert np.array_equal(to_host(lcp), eager[1]), f"replay {rep} lcp"
        # eager work of the program between replays
        gpu_sort(c[: int(o[100])], o[:101], ctx=ctx)
    g.close()


def test_graph_sees_new_contents():
    """Same buffers, new string contents: the replay sorts the new data."""
    import paper_1808_00963_amd as ss
    note("case graph new contents")
    c1, o1 = gen.generate("random", 30000, 1)
    rng = np.random.default_rng(3)
    c2 = rng.integers(ord("a"), ord("e"), len(c1), dtype=np.uint8)
    sb = np.array([0, 10000, 30000], dtype=np.uint32)
    ctx = ss.Context()
    cd, od = to_device(c1, o1)
    sbd = torch.from_numpy(sb.astype(np.int32)).cuda()
    perm = torch.empty(30000, dtype=torch.int32, device="cuda")
    lcp = torch.empty_like(perm)
    g = ctx.graph_batch(cd, od, sbd, perm, lcp)
    g.launch()
    ctx.sync()
    check_sets(c1, o1, sb, to_host(perm), to_host(lcp))
    cd.copy_(torch.from_numpy(c2).cuda())
    g.launch()
    ctx.sync()
    check_sets(c2, o1, sb, to_host(perm), to_host(lcp))
    g.close()


def test_bad_set_boundaries():
    import paper_1808_00963_amd as ss
    c, o = gen.generate("random", 1000, 1)
    cd, od = to_device(c, o)
    ctx = ss.Context()
    bad = torch.tensor([0, 600, 500, 1000], dtype=torch.int32, device="cuda")
    ctx.sort_batch(cd, od, bad)
    with pytest.raises(ss.SSError) as e:
        ctx.sync()
    assert e.value.status == ss.SS_INVALID_ARG


@pytest.mark.parametrize("mode", MODES)
def test_full_batched_workload(mode):
    """4096 sets, character budgets log-uniform in [1e3, 1e6]."""
    import paper_1808_00963_amd as ss
    note(f"case full batched mode={mode}")
    c, o, sb = gen.batch_sets()
    ctx = ss.Context()
    ctx.set_config(mode=mode)
    p, l = run_batch(c, o, sb, ctx)
    check_sets(c, o, sb, p, l, full=False)


def test_autotune_batch_and_cache():
    """The autotuner leaves the batch's correct result in the outputs, picks
    a configuration from its grid and answers a repeat from its cache."""
    import paper_1808_00963_amd as ss
    note("case autotune batch")
    ss.autotune_clear_cache()
    c, o, sb = small_batch(num_sets=40, seed=31)
    cd, od = to_device(c, o)
    sbd = torch.from_numpy(sb.astype(np.int32)).cuda()
    ctx = ss.Context()
    cfg, ms, p, l = ctx.autotune(cd, od, sbd, reps=1)
    torch.cuda.synchronize()
    check_sets(c, o, sb, to_host(p), to_host(l))
    assert cfg["max_log_splitters"] in (8, 9, 10) and cfg["bucket_target"] in (32, 64, 128)
    assert cfg["base_max"] in (512, 1024) and ms > 0
    assert {f: int(getattr(ctx.config, f)) for f in cfg} == cfg
    cfg2, ms2, p2, l2 = ctx.autotune(cd, od, sbd, reps=1)
    torch.cuda.synchronize()
    assert cfg2 == cfg and ms2 == ms
    assert np.array_equal(to_host(p2), to_host(p)) and np.array_equal(to_host(l2), to_host(l))


def test_autotune_single_set():
    import paper_1808_00963_amd as ss
    note("case autotune single")
    c, o = gen.generate("urls", 20000, 12)
    cd, od = to_device(c, o)
    ctx = ss.Context()
    cfg, ms, p, l = ctx.autotune(cd, od, reps=1, use_cache=False)
    torch.cuda.synchronize()
    assert_equal_to_oracle(c, o, to_host(p), to_host(l), label="autotune single")


def test_first_level_sampling_beside_the_gather():
    """From 2^21 strings on, the first level's sampling reads its keys from
    the strings on a second stream while the key gather runs: sets of every
    kind around it (empty, one string, base-case sizes, just above the
    base-case bound, large) and plain sorts on both sides of the bound."""
    import paper_1808_00963_amd as ss
    note("case fork batch")
    n = (1 << 21) + 3000
    c, o = gen.generate("markov", n, 41)
    rng = np.random.default_rng(41)
    sizes = [0, 1, 1, 2, 0, 64, 65, 1024, 1025, 1100, 5000, 70000]
    sizes += list(rng.integers(0, 3000, 40))
    sizes.append(n - sum(sizes))
    sb = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)
    ctx = ss.Context()
    p, l = run_batch(c, o, sb, ctx)
    check_sets(c, o, sb, p, l)
    for m in ((1 << 21) - 1, 1 << 21):
        note(f"case fork plain n={m}")
        cm, om = c[:int(o[m])], o[:m + 1]
        pm, lm = gpu_sort(cm, om, ctx=ctx)
        assert_equal_to_oracle(cm, om, pm, lm, label=f"n={m}")


def test_full_batched_graph():
    """The 4096-set workload as one graph: level launches plus the
    persistent tail; two replays each equal the oracle on every set."""
    import paper_1808_00963_amd as ss
    note("case full batched graph")
    c, o, sb = gen.batch_sets()
    cd, od = to_device(c, o)
    sbd = torch.from_numpy(sb.astype(np.int32)).cuda()
    n = len(o) - 1
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    lcp = torch.empty_like(perm)
    ctx = ss.Context()
    g = ctx.graph_batch(cd, od, sbd, perm, lcp)
    for rep in range(2):
        perm.fill_(-1)
        lcp.fill_(-1)
        g.launch()
        ctx.sync()
        check_sets(c, o, sb, to_host(perm), to_host(lcp), full=False)
    g.close()


def test_graph_tail_runs_deeper_contents():
    """A graph sized on shallow contents replayed on contents that need more
    levels: the persistent tail runs the extra levels."""
    import paper_1808_00963_amd as ss
    note("case graph deeper contents")
    n = 20000
    rng = np.random.default_rng(5)
    # shallow: random letters; deep: one shared 200-byte prefix, then random
    L = 220
    shallow = rng.integers(ord("a"), ord("z") + 1, n * L, dtype=np.uint8)
    deep = shallow.copy().reshape(n, L)
    deep[:, :200] = ord("p")
    deep = deep.reshape(-1)
    o = np.arange(n + 1, dtype=np.uint64) * L
    sb = np.array([0, n // 2, n], dtype=np.uint32)
    cd, od = to_device(shallow, o)
    sbd = torch.from_numpy(sb.astype(np.int32)).cuda()
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    lcp = torch.empty_like(perm)
    ctx = ss.Context()
    g = ctx.graph_batch(cd, od, sbd, perm, lcp)
    few = g.levels
    cd.copy_(torch.from_numpy(deep).cuda())
    g.launch()
    ctx.sync()
    check_sets(deep, o, sb, to_host(perm), to_host(lcp))
    eager = ss.Context()
    eager.sort_batch(cd, od, sbd)
    torch.cuda.synchronize()
    assert eager.stats()["levels"] > few
    g.close()


def shared_prefix_batch(seed=41):
    """Sets whose large equality buckets share long prefixes (so they skip
    words) beside ordinary sets; one set of exact duplicates."""
    rng = np.random.default_rng(seed)
    strings, sb = [], [0]
    for j in range(12):
        if j % 3 == 0:  # ordinary Markov set
            c, o = gen.generate("markov", int(rng.integers(500, 4000)), int(rng.integers(1, 1 << 30)))
            strings += gen.to_list(c, o)
        elif j % 3 == 1:  # a shared prefix of 40-120 characters, then short tails
            pre = bytes(rng.integers(ord("a"), ord("z"), int(rng.integers(40, 120)), dtype=np.uint8))
            for _ in range(int(rng.integers(1500, 5000))):
                strings.append(pre + bytes(rng.integers(ord("a"), ord("d"), int(rng.integers(0, 10)), dtype=np.uint8)))
        else:  # groups, each with a prefix of its own behind a common one
            for _ in range(4):
                pre = b"http://" + bytes(rng.integers(ord("a"), ord("z"), int(rng.integers(20, 80)), dtype=np.uint8))
                for _ in range(int(rng.integers(1100, 1600))):
                    strings.append(pre + bytes(rng.integers(ord("a"), ord("c"), int(rng.integers(0, 8)), dtype=np.uint8)))
        sb.append(len(strings))
    strings += [b"y" * 90] * 3000  # exact duplicates
    sb.append(len(strings))
    c, o = gen.from_list(strings)
    return c, o, np.array(sb, dtype=np.uint32)


@pytest.mark.parametrize("mode", MODES)
def test_batch_with_shared_prefixes(mode):
    """Sets whose large equality buckets skip shared words, every mode:
    each set equals the oracle on that set."""
    import paper_1808_00963_amd as ss
    note(f"case batch shared prefixes mode={mode}")
    c, o, sb = shared_prefix_batch()
    ctx = ss.Context()
    ctx.set_config(mode=mode)
    p, l = run_batch(c, o, sb, ctx)
    check_sets(c, o, sb, p, l)


def test_graph_with_shared_prefixes():
    """The captured batched sort on sets that skip shared words: every replay
    equals the eager result, which equals the oracle."""
    import paper_1808_00963_amd as ss
    note("case graph shared prefixes")
    c, o, sb = shared_prefix_batch(seed=43)
    ctx = ss.Context()
    eager = run_batch(c, o, sb, ctx)
    check_sets(c, o, sb, *eager)
    cd, od = to_device(c, o)
    sbd = torch.from_numpy(sb.astype(np.int32)).cuda()
    n = len(o) - 1
    perm = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    lcp = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    g = ctx.graph_batch(cd, od, sbd, perm, lcp)
    stream = torch.cuda.current_stream()
    for rep in range(3):
        perm.fill_(-1)
        lcp.fill_(-1)
        g.launch(stream)
        ctx.sync(stream)
        assert np.array_equal(to_host(perm), eager[0]), f"replay {rep} perm"
        assert np.array_equal(to_host(lcp), eager[1]), f"replay {rep} lcp"
    g.close()
