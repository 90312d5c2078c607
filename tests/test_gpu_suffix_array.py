"""Parity of the HIP suffix array by prefix doubling (section 8.2,
Observation 8.1, Algorithm 8.1) with the oracle, on the GPU.

The suffix array of a text is unique, so the HIP result is compared element
by element with the oracle's (a comparison sort of the suffixes, pinned to
Figures 5.1 and 8.1).  The inverse array must be its inverse, and the number
of sorting rounds must be the one prefix doubling needs: round r resolves
depth W0 * 2^r, and the suffixes are all distinct from depth maxLCP + 1 on.
W0, the first round's window, is 32 characters, or 128 / b characters for a
text of sigma <= 16 distinct bytes, b = 1, 2 or 4 bits per character, the
smallest that holds sigma ranks (alphabet compression).
"""
import sys

import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import needs_gpu, to_host
from pins import read_golden

pytestmark = [pytest.mark.gpu, needs_gpu]

def first_window(text):
    sigma = len(set(bytes(text)))
    b = 1
    while (1 << b) < sigma:
        b *= 2
    return 128 // b if b <= 4 else 32


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_1808_00963_amd as ss
    return ss.Context()


def gpu_sa(ctx, text):
    t = torch.from_numpy(np.ascontiguousarray(text, dtype=np.uint8)).cuda()
    sa, isa, rounds = ctx.suffix_array(t)
    torch.cuda.synchronize()
    return to_host(sa), to_host(isa), rounds


def expected_rounds(text, sa):
    """Rounds prefix doubling needs: the first r with W0 * 2^r > max LCP of
    suffixes adjacent in the suffix array."""
    t = bytes(text)
    w0 = first_window(t)
    m = 0
    for a, b in zip(sa[:-1], sa[1:]):
        x, y = t[a:], t[b:]
        k = 0
        while k < len(x) and k < len(y) and x[k] == y[k]:
            k += 1
        m = max(m, k)
    r = 0
    while w0 << r <= m:
        r += 1
    return r + 1


def check(ctx, text, label, rounds=True):
    n = len(text)
    sa, isa, r = gpu_sa(ctx, text)
    want = oracle.suffix_array(text)
    bad = np.nonzero(sa != want)[0]
    assert bad.size == 0, f"{label}: SA differs at {bad[:10]} (of {bad.size})"
    inv = np.empty(n, dtype=np.uint32)
    inv[want.astype(np.int64)] = np.arange(n, dtype=np.uint32)
    assert np.array_equal(isa, inv), f"{label}: ISA is not the inverse suffix array"
    if rounds:
        assert r == expected_rounds(text, want), f"{label}: {r} rounds"
    return r


def test_figure_8_1(ctx):
    g = read_golden("fig81_prefix_doubling.txt")
    t = np.frombuffer(g["text"].encode(), dtype=np.uint8)
    sa, isa, r = gpu_sa(ctx, t)
    assert sa.tolist() == [int(x) for x in g["sa"].split()]
    assert r == 1  # every suffix is distinct within the first window


def test_figure_5_1(ctx):
    g = read_golden("fig51_suffix_array.txt")
    t = np.frombuffer(g["text"].encode(), dtype=np.uint8)
    sa, _, _ = gpu_sa(ctx, t)
    assert sa.tolist() == [int(x) for x in g["sa"].split()][1:]  # the figure's empty suffix is not a suffix here


@pytest.mark.parametrize("n", [1, 2, 7, 8, 9, 100, 4095, 4096, 4097, 100003])
@pytest.mark.parametrize("kind", ["dna", "bytes", "zipf"])
def test_texts_vs_oracle(ctx, kind, n):
    note(f"case sa kind={kind} n={n}")
    t = gen.text(kind, n, 50 + n)
    check(ctx, t, f"{kind}/{n}", rounds=n <= 4097)


@pytest.mark.parametrize("n", [100, 5000, 20000])
def test_periodic_texts(ctx, n):
    note(f"case sa periodic n={n}")
    t = gen.text("periodic", n, n)
    check(ctx, t, f"periodic/{n}", rounds=n <= 5000)


@pytest.mark.parametrize("text", [b"a" * 3000, b"ab" * 1500, b"\x00" * 999, b"\xff\x00" * 700,
                                  b"abcabcabd" * 300, bytes(range(256)) * 8, bytes(range(16)) * 300,
                                  bytes(range(17)) * 300, b"\x00\x01\x00\x00\x01" * 500],
                         ids=["unary", "ab", "zeros", "ff00", "abcabcabd", "all_bytes", "sigma16", "sigma17",
                              "zero_ranks"])
def test_repetitive_texts(ctx, text):
    note(f"case sa repetitive {text[:8]!r} n={len(text)}")
    check(ctx, np.frombuffer(text, dtype=np.uint8), repr(text[:8]))


def test_full_size_dna_2m(ctx):
    """A 2 Mi-character ACGT text with planted 1 KiB repeats (the text of the
    suffix workload), element by element against the oracle."""
    note("case sa full dna n=2^21")
    t = gen.text("dna", 1 << 21, 4)
    check(ctx, t, "dna 2M", rounds=False)


@pytest.mark.parametrize("kind,n", [("bytes", 1 << 20), ("zipf", 1 << 20), ("periodic", 100000)])
def test_large_texts(ctx, kind, n):
    note(f"case sa large kind={kind} n={n}")
    check(ctx, gen.text(kind, n, 77), f"{kind}/{n}", rounds=False)


def test_isa_may_be_omitted_and_buffers_reused(ctx):
    """The context's workspace is reused across texts of different sizes;
    the inverse array can stay internal (NULL from C)."""
    import ctypes

    import paper_1808_00963_amd as ss
    for n in (50000, 3000, 70000):
        t = gen.text("dna", n, n)
        td = torch.from_numpy(t).cuda()
        sa = torch.empty(n, dtype=torch.int32, device="cuda")
        st = ss.lib().ss_suffix_array(ctx._h, ctypes.c_void_p(td.data_ptr()), n, ctypes.c_void_p(sa.data_ptr()),
                                      None, None, None)
        assert st == ss.SS_OK
        torch.cuda.synchronize()
        assert np.array_equal(to_host(sa), oracle.suffix_array(t)), f"n={n}"


def test_empty_text_and_context_reuse(ctx):
    import paper_1808_00963_amd as ss
    sa, isa, r = ctx.suffix_array(torch.zeros(0, dtype=torch.uint8, device="cuda"))
    assert sa.numel() == 0 and r == 0
    # the same context sorts strings afterwards
    c, o = gen.generate("markov", 5000, 3)
    from gpu_util import assert_equal_to_oracle, gpu_sort
    p, l = gpu_sort(c, o, ctx=ctx)
    assert_equal_to_oracle(c, o, p, l)
    assert ctx.last_error() == ss.SS_OK


def test_plain_sort_after_a_large_suffix_array():
    """One context: a suffix array of 2^21 characters (its sorts run with a
    bucket target of at least 256 and host-read level counts), then plain
    sorts of 2^21 and 2^22 Markov strings, which need the pools of the
    default bucket target of 64 and the device-driven levels: both equal to
    the oracle, and the context reports no error."""
    import paper_1808_00963_amd as ss
    from gpu_util import assert_equal_to_oracle, gpu_sort
    note("case sa then plain sorts")
    c2 = ss.Context()
    t = gen.text("dna", 1 << 21, 9)
    sa, _, _ = gpu_sa(c2, t)
    assert np.array_equal(sa, oracle.suffix_array(t))
    for n in (1 << 21, 1 << 22):
        c, o = gen.generate("markov", n, 3)
        p, l = gpu_sort(c, o, ctx=c2)
        assert_equal_to_oracle(c, o, p, l, full=False, label=f"markov {n} after the suffix array")
    assert c2.last_error() == ss.SS_OK
    cfg = c2.config
    assert cfg.bucket_target == 64 and cfg.mode == ss.MODE_LEVELS
