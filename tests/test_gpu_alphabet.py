"""Alphabet-compressed keys (alphabet compression, section 4.6.1) on the
GPU.  With alphabet="compress" inputs of 1..15 distinct bytes are sorted
with 32, 21 or 16 characters per key; with "auto" (the default) inputs of at
most 3 distinct bytes and at most 64 characters per string on average; every
other input with byte keys.  Either way the result equals the oracle's, and
equals the byte-key sort of the same input."""
import sys

import numpy as np
import pytest

import gen
from gpu_util import assert_equal_to_oracle, gpu_sort, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def strings_over(alphabet: bytes, n: int, seed: int, max_len=70, shared=0):
    """Random strings over `alphabet`; with `shared`, a fraction of them
    start with one of a few long common prefixes (deep ties)."""
    rng = np.random.default_rng(seed)
    syms = np.frombuffer(alphabet, dtype=np.uint8)
    prefixes = [bytes(rng.choice(syms, rng.integers(20, 60))) for _ in range(4)]
    out = []
    for i in range(n):
        s = bytes(rng.choice(syms, rng.integers(0, max_len)))
        if shared and rng.random() < shared:
            s = prefixes[rng.integers(0, 4)] + s[: rng.integers(0, 30)]
        out.append(s)
    return out


def sort_with(strings, alphabet_mode):
    import paper_1808_00963_amd as ss
    c, o = gen.from_list(strings)
    ctx = ss.Context()
    ctx.set_config(alphabet=alphabet_mode)
    p, l = gpu_sort(c, o, ctx=ctx)
    return c, o, p, l, ctx.stats()


@pytest.mark.parametrize("alphabet,key_chars", [
    (b"a", 32), (b"ab", 32), (b"\x00\xff", 32), (b"xyz", 32), (b"ACGT", 21), (b"ACGTN\x00\x01", 21),
    (bytes(range(200, 208)), 16), (bytes(range(0, 240, 16)), 16), (bytes(range(64, 80)), 8)])
@pytest.mark.parametrize("n", [777, 20000])
def test_alphabets_vs_oracle(alphabet, key_chars, n):
    note(f"case alphabet={alphabet!r} n={n}")
    strings = strings_over(alphabet, n, 31 + n, shared=0.3)
    c, o, p, l, st = sort_with(strings, "compress")
    assert_equal_to_oracle(c, o, p, l, label=f"{alphabet!r}/{n}")
    assert st["key_chars"] == key_chars
    if key_chars != 8:
        assert st["alphabet_size"] == len(set(alphabet))


def test_rare_byte_beyond_the_probe():
    """A fifth symbol in a few strings, after the 16 bytes the probe reads
    but inside every string's first key: the first attempt's key gather
    meets it, the sort runs again with the full check, which finds the
    fifth symbol; keys stay compressed (21 per key)."""
    note("case rare byte")
    strings = strings_over(b"ACGT", 30000, 5, max_len=100)
    for i in range(7, 30000, 4999):
        s = strings[i]
        strings[i] = (s + b"ACGTACGTACGTACGTACGTACGT")[:17] + b"N" + s[17:]
    c, o, p, l, st = sort_with(strings, "compress")
    assert_equal_to_oracle(c, o, p, l, label="rare byte")
    assert st["key_chars"] == 21 and st["alphabet_size"] == 5
    assert st["alphabet_retries"] == 1


def test_byte_the_sort_never_reads():
    """A fourth symbol only far inside strings that differ from every other
    string within their first key: no gather reads it, so the first attempt
    (keys compressed with the three probed symbols, 32 per key) stands and
    still equals the oracle."""
    note("case unread byte")
    strings = strings_over(b"ACG", 30000, 8, max_len=100)
    heads = {}
    for s in strings:
        heads[s[:32]] = heads.get(s[:32], 0) + 1
    marked = 0
    for i in range(11, 30000, 331):
        s = strings[i]
        if len(s) > 70 and heads[s[:32]] == 1:  # no other string shares its first key
            strings[i] = s[:60] + b"T" + s[61:]
            marked += 1
    assert marked >= 10
    c, o, p, l, st = sort_with(strings, "compress")
    assert_equal_to_oracle(c, o, p, l, label="unread byte")
    assert st["alphabet_retries"] == 0
    assert st["key_chars"] == 32 and st["alphabet_size"] == 3


def test_too_many_bytes_after_the_probe():
    """Fifteen symbols in the strings' first bytes, more later: some strings
    share their first key (16 characters) and differ in a byte outside the
    probed set, the gather one key further meets it, and the check of the
    second attempt gives up: byte keys."""
    note("case over")
    syms = bytes(range(97, 112))
    strings = strings_over(syms, 20000, 6, max_len=60)
    head = bytes(syms[(7 * k) % 15] for k in range(16))
    for i in range(3, 20000, 97):
        strings[i] = head + bytes([200 + (i % 30)]) + strings[i][:20]
    c, o, p, l, st = sort_with(strings, "compress")
    assert_equal_to_oracle(c, o, p, l, label="over")
    assert st["key_chars"] == 8 and st["alphabet_retries"] == 1


@pytest.mark.parametrize("model", ["binary", "dna_reads"])
def test_bytes_setting_gives_the_same_result(model):
    note(f"case same result {model}")
    if model == "binary":
        c, o = gen.generate(model, 40000, 9)
        strings = [bytes(c[int(o[i]):int(o[i + 1])]) for i in range(len(o) - 1)]
    else:  # 50-character windows of the suffix workload's DNA text
        t = gen.text("dna", 60000, 9)
        strings = [bytes(t[i:i + 50]) for i in range(0, 59000, 3)]
    c, o, p1, l1, s1 = sort_with(strings, "auto" if model == "binary" else "compress")
    _, _, p2, l2, s2 = sort_with(strings, "bytes")
    assert np.array_equal(p1, p2) and np.array_equal(l1, l2)
    assert s2["key_chars"] == 8 and s1["key_chars"] > 8
    assert_equal_to_oracle(c, o, p1, l1, label=model)


def test_auto_policy():
    """"auto" compresses short strings of at most 3 distinct bytes only:
    two symbols, short: 32 characters per key; four symbols, short, or two
    symbols and more than 64 characters per string on average: byte keys
    (the same inputs with "compress" get 21 / 32)."""
    cases = [(strings_over(b"ab", 20000, 1, max_len=60), 32, 32),
             (strings_over(b"ACGT", 20000, 2, max_len=60), 8, 21),
             ([s * 4 for s in strings_over(b"ab", 5000, 3, max_len=60)], 8, 32)]
    for k, (strings, auto_chars, compress_chars) in enumerate(cases):
        note(f"case auto policy {k}")
        c, o, p, l, st = sort_with(strings, "auto")
        assert_equal_to_oracle(c, o, p, l, label=f"auto {k}")
        assert st["key_chars"] == auto_chars
        c, o, p2, l2, st2 = sort_with(strings, "compress")
        assert np.array_equal(p, p2) and np.array_equal(l, l2)
        assert st2["key_chars"] == compress_chars


@pytest.mark.parametrize("mode", ["levels", "host_levels", "persistent"])
@pytest.mark.parametrize("form", ["single", "batch"])
def test_retry_in_every_mode_and_in_a_batch(mode, form):
    """A symbol outside the probed set inside the first key of a few strings
    of one set: the level modes sort a second time with the full check
    (one retry), the persistent mode checks before its launch (none); either
    way every set equals the oracle with 5 symbols, 21 per key."""
    import paper_1808_00963_amd as ss
    import torch
    from gpu_util import to_device, to_host
    note(f"case retry mode={mode} form={form}")
    strings = strings_over(b"ACGT", 9000, 12, max_len=80, shared=0.2)
    for i in range(5003, 5400, 97):  # inside the fourth set of the batch
        s = strings[i]
        strings[i] = (s + b"TTGCATTGCATTGCATTGCA")[:18] + b"N" + s[18:]
    c, o = gen.from_list(strings)
    ctx = ss.Context()
    ctx.set_config(mode=mode, alphabet="compress")
    if form == "single":
        p, l = gpu_sort(c, o, ctx=ctx)
        assert_equal_to_oracle(c, o, p, l, label=f"{mode}")
    else:
        sb = np.array([0, 1, 1, 4000, 8999, 9000], dtype=np.uint32)
        cd, od = to_device(c, o)
        pd, ld = ctx.sort_batch(cd, od, torch.from_numpy(sb.astype(np.int32)).cuda())
        torch.cuda.synchronize()
        p, l = to_host(pd), to_host(ld)
        for j in range(len(sb) - 1):
            b, e = int(sb[j]), int(sb[j + 1])
            if e > b:
                cj = c[int(o[b]):int(o[e])]
                oj = o[b:e + 1] - o[b]
                assert_equal_to_oracle(cj, oj, p[b:e], l[b:e], label=f"{mode} set {j}")
    st = ctx.stats()
    assert st["key_chars"] == 21 and st["alphabet_size"] == 5
    assert st["alphabet_retries"] == (0 if mode == "persistent" else 1)


def test_compressed_modes_and_batch():
    """Compressed keys in the host-driven and persistent modes and in a batch
    of DNA sets."""
    import paper_1808_00963_amd as ss
    import torch
    from gpu_util import to_device, to_host
    strings = strings_over(b"ACGT", 12000, 8, shared=0.2)
    c, o = gen.from_list(strings)
    for mode in ("host_levels", "persistent"):
        note(f"case compressed mode={mode}")
        ctx = ss.Context()
        ctx.set_config(mode=mode, alphabet="compress")
        p, l = gpu_sort(c, o, ctx=ctx)
        assert_equal_to_oracle(c, o, p, l, label=mode)
        assert ctx.stats()["key_chars"] == 21
    note("case compressed batch")
    sb = np.array([0, 10, 10, 3000, 11999, 12000], dtype=np.uint32)
    cd, od = to_device(c, o)
    ctx = ss.Context()
    ctx.set_config(alphabet="compress")
    pd, ld = ctx.sort_batch(cd, od, torch.from_numpy(sb.astype(np.int32)).cuda())
    torch.cuda.synchronize()
    p, l = to_host(pd), to_host(ld)
    for j in range(len(sb) - 1):
        b, e = int(sb[j]), int(sb[j + 1])
        if e > b:
            cj = c[int(o[b]):int(o[e])]
            oj = o[b:e + 1] - o[b]
            assert_equal_to_oracle(cj, oj, p[b:e], l[b:e], label=f"set {j}")
