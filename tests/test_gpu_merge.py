"""Parity of the HIP LCP-aware merge of sorted runs (section 4.3.1,
Algorithms 4.2-4.4) with the oracle, on the GPU.

The merge of runs that hold a multiset of string indices has one correct
answer: the multiset ordered by (string, index) with its LCP array.  The
expected value is therefore the oracle's sort of the strings of that
multiset, taken in increasing index order (so the oracle's tie order by
position is the order by original index); copies of an index are identical
and adjacent.  The runs fed to the merge are sorted by the oracle too, except
in the end-to-end cases, which merge runs sorted by the HIP sort.
"""
import sys

import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import assert_equal_to_oracle, needs_gpu, to_device, to_host

pytestmark = [pytest.mark.gpu, needs_gpu]

TILE = 2048  # outputs per work group of the merge kernel (8 per thread)


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def subset(chars, offsets, idx):
    """(chars, offsets) of the strings idx (in the given order)."""
    s = gen.to_list(chars, offsets)
    return gen.from_list([s[i] for i in idx])


def oracle_sorted(chars, offsets, idx):
    """(perm, lcp) of the multiset idx of strings, ordered by (string, index)."""
    idx = np.sort(np.asarray(idx, dtype=np.int64))
    if idx.size == 0:
        return np.zeros(0, np.uint32), np.zeros(0, np.uint32)
    c, o = subset(chars, offsets, idx)
    p, l = oracle.sort(c, o)
    return idx[p.astype(np.int64)].astype(np.uint32), l


def make_runs(chars, offsets, parts):
    """Concatenated oracle-sorted runs of the index lists `parts`."""
    perm, lcp, rb = [], [], [0]
    for part in parts:
        p, l = oracle_sorted(chars, offsets, part)
        if l.size:
            l = l.copy()
            l[0] = 0xDEADBEEF  # a run's first LCP entry is not read
        perm.append(p)
        lcp.append(l)
        rb.append(rb[-1] + len(part))
    cat = lambda xs: np.concatenate(xs) if xs else np.zeros(0, np.uint32)
    return cat(perm).astype(np.uint32), cat(lcp).astype(np.uint32), rb


def dev_u32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def gpu_merge(ctx, chars, offsets, perm, lcp, rb):
    c, o = to_device(chars, offsets)
    p, l = ctx.merge_runs(c, o, dev_u32(perm), dev_u32(lcp), rb)
    torch.cuda.synchronize()
    return to_host(p), to_host(l)


def check_merge(ctx, chars, offsets, parts, label):
    perm, lcp, rb = make_runs(chars, offsets, parts)
    got_p, got_l = gpu_merge(ctx, chars, offsets, perm, lcp, rb)
    want_p, want_l = oracle_sorted(chars, offsets, np.concatenate([np.asarray(x, np.int64) for x in parts]))
    bad_p = np.nonzero(got_p != want_p)[0]
    bad_l = np.nonzero(got_l != want_l)[0]
    assert bad_p.size == 0, f"{label}: perm differs at {bad_p[:10]} (of {bad_p.size})"
    assert bad_l.size == 0, f"{label}: lcp differs at {bad_l[:10]}: got {got_l[bad_l[:10]]} want {want_l[bad_l[:10]]}"


def random_partition(n, k, seed):
    rng = np.random.default_rng(seed)
    owner = rng.integers(0, k, n)
    return [np.nonzero(owner == r)[0] for r in range(k)]


@pytest.fixture(scope="module")
def ctx():
    import paper_1808_00963_amd as ss
    return ss.Context()


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 17])
@pytest.mark.parametrize("n", [1, 2, 9, 1000, TILE - 1, TILE, TILE + 1, 20000])
@pytest.mark.parametrize("model", ["random", "binary", "markov", "urls"])
def test_partition_merge_vs_oracle(ctx, model, n, k):
    note(f"case merge model={model} n={n} k={k}")
    c, o = gen.generate(model, n, 300 + n + k)
    check_merge(ctx, c, o, random_partition(n, k, 7 * n + k), f"{model}/{n}/{k}")


@pytest.mark.parametrize("n", [3000, 20000])
def test_suffix_runs(ctx, n):
    note(f"case merge suffixes n={n}")
    c, o = gen.generate("suffixes", n, 11)
    check_merge(ctx, c, o, random_partition(n, 4, n), f"suffixes/{n}")


def test_contiguous_halves_and_ragged_sizes(ctx):
    c, o = gen.generate("markov", 100003, 21)
    for cut in (0, 1, 8, TILE, 50000, 100002, 100003):
        note(f"case merge halves cut={cut}")
        check_merge(ctx, c, o, [np.arange(cut), np.arange(cut, 100003)], f"cut={cut}")


def test_empty_runs_and_single_element_runs(ctx):
    c, o = gen.generate("urls", 600, 5)
    parts = [[], np.arange(0, 200), [], [], np.arange(200, 201), np.arange(201, 600), []]
    note("case merge empty runs")
    check_merge(ctx, c, o, parts, "empty runs")
    note("case merge one element per run")
    check_merge(ctx, c, o, [[i] for i in np.random.default_rng(3).permutation(600)], "singletons")


def test_all_runs_empty_is_a_no_op(ctx):
    c, o = gen.generate("random", 10, 1)
    perm, lcp, rb = make_runs(c, o, [[], []])
    cd, od = to_device(c, o)
    out_p = torch.full((4,), 7, dtype=torch.int32, device="cuda")
    out_l = torch.full((4,), 7, dtype=torch.int32, device="cuda")
    ctx.merge_runs(cd, od, torch.zeros(1, dtype=torch.int32, device="cuda"),
                   torch.zeros(1, dtype=torch.int32, device="cuda"), rb, out_p, out_l)
    assert to_host(out_p).tolist() == [7] * 4


def test_duplicate_indices_across_runs(ctx):
    c, o = gen.generate("markov", 3000, 9)
    rng = np.random.default_rng(4)
    parts = [rng.integers(0, 3000, 1500), rng.integers(0, 3000, 2000), np.arange(3000), rng.integers(0, 50, 300)]
    note("case merge duplicates")
    check_merge(ctx, c, o, parts, "duplicates")


def _adversarial():
    rng = np.random.default_rng(5)
    base = bytes(rng.integers(0, 256, 600, dtype=np.uint8))
    return {
        "all_equal": [b"abcdefghij"] * 3000,
        "all_empty": [b""] * 2000,
        "empty_and_zero_bytes": [b"", b"\x00", b"\x00\x00", b"", b"\x00\xff", b"\xff", b"\x00"] * 300,
        "nested_prefixes": [b"a" * k for k in range(600, 0, -1)],
        "long_common_prefix": [base[:512] + bytes([x]) for x in rng.integers(0, 3, 4000)],
        "prefix_ladder": [base[:k] for k in rng.integers(0, 520, 5000)],
    }


@pytest.mark.parametrize("name", sorted(_adversarial()))
@pytest.mark.parametrize("k", [2, 7])
def test_adversarial_runs(ctx, name, k):
    note(f"case merge adversarial {name} k={k}")
    c, o = gen.from_list(_adversarial()[name])
    n = len(o) - 1
    check_merge(ctx, c, o, random_partition(n, k, n + k), name)


def test_merge_of_gpu_sorted_halves_equals_gpu_sort(ctx):
    """End to end: the HIP batched sort sorts two halves, the merge joins them."""
    for model, n in (("markov", 200000), ("urls", 50001), ("suffixes", 20000)):
        note(f"case merge e2e model={model} n={n}")
        c, o = gen.generate(model, n, 17)
        cd, od = to_device(c, o)
        h = n // 2
        sb = torch.tensor([0, h, n], dtype=torch.int32, device="cuda")
        p, l = ctx.sort_batch(cd, od, sb)
        p[h:] += h  # set-local -> global string index
        mp, ml = ctx.merge_runs(cd, od, p, l, [0, h, n])
        torch.cuda.synchronize()
        assert_equal_to_oracle(c, o, to_host(mp), to_host(ml), label=f"e2e/{model}")


@pytest.mark.parametrize("seed", range(6))
def test_random_run_counts(ctx, seed):
    """K from 2 to 64 runs of random sizes over a random model and size."""
    rng = np.random.default_rng(700 + seed)
    model = ["random", "markov", "urls", "binary", "bytes"][seed % 5]
    n = int(rng.integers(1000, 40000))
    k = int(rng.integers(2, 65))
    note(f"case merge random runs seed={seed} model={model} n={n} k={k}")
    c, o = gen.generate(model, n, 900 + seed)
    check_merge(ctx, c, o, random_partition(n, k, seed), f"seed {seed}")


def test_many_gpu_sorted_runs_equal_gpu_sort(ctx):
    """End to end with 37 runs: the batched sort sorts 37 contiguous sets,
    the merge joins them; equals the oracle's sort of the whole set."""
    c, o = gen.generate("urls", 120000, 23)
    n = len(o) - 1
    cd, od = to_device(c, o)
    rb = [n * r // 37 for r in range(38)]
    sb = torch.tensor(rb, dtype=torch.int32, device="cuda")
    p, l = ctx.sort_batch(cd, od, sb)
    for r in range(37):
        p[rb[r]:rb[r + 1]] += rb[r]
    mp, ml = ctx.merge_runs(cd, od, p, l, rb)
    torch.cuda.synchronize()
    assert_equal_to_oracle(c, o, to_host(mp), to_host(ml), label="37 runs")


def test_full_size_c1_halves(ctx):
    """16M Markov strings: sorted halves merged, verified by the oracle's
    linear-time check (the answer is unique)."""
    note("case merge full c1_markov_16m halves")
    c, o = gen.workload("c1_markov_16m")
    n = len(o) - 1
    cd, od = to_device(c, o)
    h = n // 2
    sb = torch.tensor([0, h, n], dtype=torch.int32, device="cuda")
    p, l = ctx.sort_batch(cd, od, sb)
    p[h:] += h
    mp, ml = ctx.merge_runs(cd, od, p, l, [0, h, n])
    torch.cuda.synchronize()
    assert_equal_to_oracle(c, o, to_host(mp), to_host(ml), full=False, label="c1 halves")


def test_argument_errors(ctx):
    import paper_1808_00963_amd as ss
    c, o = gen.generate("random", 100, 2)
    perm, lcp, rb = make_runs(c, o, random_partition(100, 3, 1))
    cd, od = to_device(c, o)
    pd, ld = dev_u32(perm), dev_u32(lcp)
    for bad in ([1, 50, 100], [0, 60, 50, 100]):
        with pytest.raises(ss.SSError) as e:
            ctx.merge_runs(cd, od, pd, ld, bad)
        assert e.value.status == ss.SS_INVALID_ARG
    with pytest.raises(ss.SSError) as e:
        ctx.merge_runs(cd, od, pd, ld, rb, perm_out=pd)
    assert e.value.status == ss.SS_INVALID_ARG


def test_index_out_of_range_is_an_error_and_context_recovers(ctx):
    import paper_1808_00963_amd as ss
    note("case merge index out of range")
    c, o = gen.generate("markov", 1000, 3)
    perm, lcp, rb = make_runs(c, o, random_partition(1000, 2, 3))
    bad = perm.copy()
    bad[rb[1] // 2] = 1000  # one past the last string
    cd, od = to_device(c, o)
    with pytest.raises(ss.SSError) as e:
        ctx.merge_runs(cd, od, dev_u32(bad), dev_u32(lcp), rb)
        torch.cuda.synchronize()
    assert e.value.status == ss.SS_INVALID_ARG
    check_merge(ctx, c, o, random_partition(1000, 2, 3), "after error")
