"""Pins for the oracle: checks against results fixed by the paper or by
mathematics, independent of the oracle's own code.

Each function takes an oracle library handle (so the mutation test can run
the same pins against deliberately broken builds of the oracle) and returns a
list of failure descriptions (empty = pinned).
"""
from __future__ import annotations

import itertools
import os
import random

import numpy as np

import gen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def read_golden(name):
    out = {}
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split(":", 1)
                out[k.strip()] = v.strip()
    return out


def lcp_py(a: bytes, b: bytes) -> int:
    k = 0
    while k < len(a) and k < len(b) and a[k] == b[k]:
        k += 1
    return k


def expected_by_library(strings):
    """Python's built-in sort of (bytes, index) pairs: bytes compare as
    unsigned values with a proper prefix smaller."""
    perm = sorted(range(len(strings)), key=lambda i: (strings[i], i))
    lcp = [0] + [lcp_py(strings[perm[k - 1]], strings[perm[k]]) for k in range(1, len(perm))]
    return perm, lcp


def insertion_sort_textbook(strings):
    """String insertion sort in the manner of Algorithm 2.5 (section 2.2.5),
    with explicit lengths instead of terminators and ties kept in index
    order (the insertion stops at an equal string, so it is stable)."""
    def less(x, y):  # x < y by characters, then length
        p = 0
        while p < len(x) and p < len(y) and x[p] == y[p]:
            p += 1
        if p < len(x) and p < len(y):
            return x[p] < y[p]
        return len(x) < len(y)

    order = list(range(len(strings)))
    for i in range(1, len(order)):
        x = order[i]
        j = i
        while j > 0 and less(strings[x], strings[order[j - 1]]):
            order[j] = order[j - 1]
            j -= 1
        order[j] = x
    return order


def suffix_array_doubling(text: bytes):
    """Suffix array by prefix doubling (Manber-Myers style: sort by rank
    pairs (r[i], r[i+k]) for k = 1, 2, 4, ...), section 5.2."""
    n = len(text)
    rank = list(text)
    sa = list(range(n))
    k = 1
    while True:
        key = lambda i: (rank[i], rank[i + k] if i + k < n else -1)
        sa.sort(key=key)
        new = [0] * n
        for t in range(1, n):
            new[sa[t]] = new[sa[t - 1]] + (key(sa[t]) != key(sa[t - 1]))
        rank = new
        if n == 0 or rank[sa[-1]] == n - 1:
            return sa
        k *= 2


def kasai_lcp(text: bytes, sa):
    """LCP array from text and suffix array (Kasai et al.), section 5.6."""
    n = len(text)
    rank = [0] * n
    for i, s in enumerate(sa):
        rank[s] = i
    lcp = [0] * n
    h = 0
    for i in range(n):
        if rank[i] > 0:
            j = sa[rank[i] - 1]
            while i + h < n and j + h < n and text[i + h] == text[j + h]:
                h += 1
            lcp[rank[i]] = h
            if h:
                h -= 1
        else:
            h = 0
    return lcp


def _run(lib, strings):
    c, o = gen.from_list(strings)
    p, l = oracle.sort(c, o, lib=lib)
    return p.tolist(), l.tolist()


# --------------------------------------------------------------------------
# individual pins
# --------------------------------------------------------------------------

def pin_lemma21(lib):
    g = read_golden("lemma21_example.txt")
    strings = [s.encode() for s in g["strings"].split()]
    p, l = _run(lib, strings)
    fails = []
    if p != [int(x) for x in g["perm"].split()]:
        fails.append(f"lemma 2.1 example perm {p}")
    if l != [int(x) for x in g["lcp"].split()]:
        fails.append(f"lemma 2.1 example lcp {l}")
    if sum(l[1:]) != int(g["L"]):
        fails.append("lemma 2.1 example L")
    return fails


def pin_fig51(lib):
    g = read_golden("fig51_suffix_array.txt")
    t = g["text"].encode()
    strings = [t[i:] for i in range(len(t) + 1)]
    p, l = _run(lib, strings)
    fails = []
    if p != [int(x) for x in g["sa"].split()]:
        fails.append(f"figure 5.1 SA {p}")
    if l != [int(x) for x in g["lcp"].split()]:
        fails.append(f"figure 5.1 LCP {l}")
    return fails


def pin_library_sort(lib, seeds=range(6)):
    fails = []
    for seed in seeds:
        rng = random.Random(seed)
        n = rng.choice([1, 2, 3, 17, 200, 1000])
        alphabet = rng.choice([b"ab", b"\x00\xff", bytes(range(256)), b"a\x00b\xff"])
        maxlen = rng.choice([0, 1, 3, 9, 20])
        strings = [bytes(rng.choice(alphabet) for _ in range(rng.randint(0, maxlen))) for _ in range(n)]
        if rng.random() < 0.5 and n > 2:  # duplicates and nested prefixes
            strings[rng.randrange(n)] = strings[0]
            strings[rng.randrange(n)] = strings[0] + b"\x00"
        exp = expected_by_library(strings)
        got = _run(lib, strings)
        if got != (exp[0], exp[1]):
            fails.append(f"library-sort mismatch seed {seed}")
    for model in ("bytes", "binary", "urls"):
        c, o = gen.generate(model, 700, 11)
        strings = gen.to_list(c, o)
        if _run(lib, strings) != expected_by_library(strings):
            fails.append(f"library-sort mismatch model {model}")
    return fails


def pin_exhaustive(lib):
    """All strings of length <= 3 over {0x00, 'a', 'b', 0xFF}, each twice,
    shuffled; the expected order is the enumeration order itself."""
    alpha = [0x00, ord("a"), ord("b"), 0xFF]
    universe = [b""]
    for L in (1, 2, 3):
        universe += [bytes(t) for t in itertools.product(alpha, repeat=L)]
    universe.sort()  # lexicographic by unsigned bytes, prefix first
    strings = universe + universe
    idx = list(range(len(strings)))
    random.Random(7).shuffle(idx)
    shuffled = [strings[i] for i in idx]
    p, l = _run(lib, shuffled)
    fails = []
    # sorted sequence must be every string twice, in universe order
    if [shuffled[i] for i in p] != [u for u in universe for _ in (0, 1)]:
        fails.append("exhaustive order")
    # equal strings by index
    for k in range(1, len(p)):
        if shuffled[p[k]] == shuffled[p[k - 1]] and p[k] < p[k - 1]:
            fails.append("exhaustive tie order")
            break
    for k in range(1, len(p)):
        a, b = shuffled[p[k - 1]], shuffled[p[k]]
        if l[k] != lcp_py(a, b):
            fails.append("exhaustive lcp")
            break
    return fails


def pin_insertion_sort(lib):
    fails = []
    for seed in range(20):
        rng = random.Random(100 + seed)
        strings = [bytes(rng.choice(b"ab\x00") for _ in range(rng.randint(0, 4))) for _ in range(rng.randint(1, 12))]
        if _run(lib, strings)[0] != insertion_sort_textbook(strings):
            fails.append(f"insertion-sort mismatch seed {seed}")
    return fails


def pin_truncated_suffixes(lib, tau=6):
    """Suffixes of a text truncated to tau characters, against a textbook
    suffix array (prefix doubling) plus Kasai LCP: runs of the suffix array
    with LCP >= tau hold identical truncated strings, which are ordered by
    index with LCP tau; all other neighbours keep the suffix-array order and
    LCP."""
    fails = []
    for seed in range(4):
        rng = random.Random(300 + seed)
        text = bytes(rng.choice(b"ACGT") for _ in range(rng.choice([50, 300, 800])))
        if seed % 2:  # plant repeats
            w = text[10:40]
            text = text[:100] + w + text[130:200] + w + text[230:]
        n = len(text)
        sa = suffix_array_doubling(text)
        h = kasai_lcp(text, sa)
        exp_perm, exp_lcp = [], []
        k = 0
        while k < n:
            e = k + 1
            while e < n and h[e] >= tau:
                e += 1
            run = sorted(sa[k:e])
            exp_lcp.append(0 if k == 0 else h[k])
            exp_lcp.extend([tau] * (len(run) - 1))
            exp_perm.extend(run)
            k = e
        strings = [text[i:i + tau] for i in range(n)]
        p, l = _run(lib, strings)
        if p != exp_perm or l != exp_lcp:
            fails.append(f"truncated suffixes seed {seed}")
    return fails


def pin_lemma21_bounds(lib):
    """n + L <= D <= 2L + n with D from its definition (distinguishing
    prefix, counting the terminator) computed over all pairs."""
    fails = []
    for seed in range(5):
        rng = random.Random(500 + seed)
        strings = list({bytes(rng.choice(b"abc") for _ in range(rng.randint(1, 6))) for _ in range(60)})
        rng.shuffle(strings)
        p, l = _run(lib, strings)
        n, L = len(strings), sum(l[1:])
        term = [s + b"\x00" for s in strings]
        D = 0
        for i in range(n):
            D += max(lcp_py(term[i], term[j]) + 1 for j in range(n) if j != i) if n > 1 else 1
        if not (n + L <= D <= 2 * L + n):
            fails.append(f"lemma 2.1 bounds seed {seed}: n={n} L={L} D={D}")
    return fails


def pin_fig81_names(lib):
    """Figure 8.1: the h-names at h = 1, 2, 4 and the final suffix array."""
    g = read_golden("fig81_prefix_doubling.txt")
    t = g["text"].encode()
    fails = []
    for h in (1, 2, 4):
        got = oracle.h_names(t, h, lib=lib).tolist()
        if got != [int(x) for x in g[f"isa{h}"].split()]:
            fails.append(f"figure 8.1 ISA^{h} {got}")
    sa = oracle.suffix_array(t, lib=lib).tolist()
    if sa != [int(x) for x in g["sa"].split()]:
        fails.append(f"figure 8.1 SA {sa}")
    return fails


def pin_fig51_suffix_array(lib):
    """Figure 5.1 without its sentinel: the empty suffix (first in the
    figure) is not a suffix of T[0..n)."""
    g = read_golden("fig51_suffix_array.txt")
    sa = oracle.suffix_array(g["text"].encode(), lib=lib).tolist()
    want = [int(x) for x in g["sa"].split()][1:]
    return [] if sa == want else [f"figure 5.1 SA {sa}"]


def pin_suffix_brute(lib, seeds=range(8)):
    """Tiny texts: the suffix array by Python's sort of the suffix slices and
    the h-names by counting smaller truncations; at h >= n the names are the
    inverse suffix array."""
    fails = []
    for seed in seeds:
        rng = random.Random(900 + seed)
        n = rng.choice([0, 1, 2, 5, 13, 40, 97])
        alphabet = rng.choice([b"a", b"ab", b"\x00\xff", bytes(range(256)), b"acgt"])
        t = bytes(rng.choice(alphabet) for _ in range(n))
        want = sorted(range(n), key=lambda i: t[i:])
        got = oracle.suffix_array(t, lib=lib).tolist()
        if got != want:
            fails.append(f"suffix array seed {seed}: {got} != {want}")
        for h in (1, 2, 3, 8, max(n, 1)):
            trunc = [t[i:i + h] for i in range(n)]
            names = [sum(1 for j in range(n) if trunc[j] < trunc[i]) for i in range(n)]
            got_n = oracle.h_names(t, h, lib=lib).tolist()
            if got_n != names:
                fails.append(f"h-names seed {seed} h={h}")
        inv = [0] * n
        for r, i in enumerate(want):
            inv[i] = r
        if n and oracle.h_names(t, n, lib=lib).tolist() != inv:
            fails.append(f"names at h=n are not the inverse suffix array, seed {seed}")
    return fails


def pin_sampled_helpers(lib, seeds=range(4)):
    """The pairwise helpers used by sampled checks (LCP of two strings,
    three-way (string, index) comparison) against Python's byte strings."""
    fails = []
    for seed in seeds:
        rng = random.Random(100 + seed)
        alphabet = rng.choice([b"ab", b"\x00\xff", b"a\x00b\xff", bytes(range(256))])
        strings = [bytes(rng.choice(alphabet) for _ in range(rng.randint(0, 12))) for _ in range(60)]
        strings[1] = strings[0]
        strings[2] = strings[0] + b"\x00"
        c, o = gen.from_list(strings)
        for _ in range(400):
            a, b = rng.randrange(60), rng.randrange(60)
            if oracle.lcp_of(c, o, a, b, lib=lib) != lcp_py(strings[a], strings[b]):
                fails.append(f"lcp_of({a},{b}) seed {seed}")
                break
            want = ((strings[a], a) > (strings[b], b)) - ((strings[a], a) < (strings[b], b))
            if oracle.compare(c, o, a, b, lib=lib) != want:
                fails.append(f"compare({a},{b}) seed {seed}")
                break
    return fails


def pin_multithreaded(lib, seeds=range(5)):
    """The all-cores variant of the sort against Python's sort of
    (bytes, index) pairs, for thread counts that leave ragged chunks."""
    fails = []
    for seed in seeds:
        rng = random.Random(200 + seed)
        n = rng.choice([0, 1, 2, 7, 300, 2000])
        alphabet = rng.choice([b"ab", b"\x00\xff", bytes(range(256))])
        strings = [bytes(rng.choice(alphabet) for _ in range(rng.randint(0, 10))) for _ in range(n)]
        if n > 4:
            strings[3] = strings[0]
            strings[4] = strings[0] + b"\x00"
        exp = expected_by_library(strings)
        c, o = gen.from_list(strings)
        for threads in (1, 2, 3, 5, 8):
            p, l = oracle.sort_mt(c, o, threads, lib=lib)
            if (p.tolist(), l.tolist()) != (exp[0], exp[1][:n]):
                fails.append(f"sort_mt mismatch seed {seed} threads {threads}")
    return fails


ALL_PINS = [pin_sampled_helpers, pin_multithreaded, pin_lemma21, pin_fig51, pin_library_sort, pin_exhaustive, pin_insertion_sort,
            pin_truncated_suffixes, pin_lemma21_bounds, pin_fig81_names, pin_fig51_suffix_array,
            pin_suffix_brute]


def run_all(lib):
    fails = []
    for f in ALL_PINS:
        try:
            fails += f(lib)
        except Exception as e:  # a crash counts as a failed pin
            fails.append(f"{f.__name__}: {type(e).__name__}: {e}")
    return fails
