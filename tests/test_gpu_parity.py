"""Parity of the HIP sort (through the C ABI) with the oracle, on the GPU.

Small and mid sizes are compared element by element with the oracle's own
sort; the full-size workloads are verified with the oracle's linear-time
check (permutation + strict (string, index) order + brute-force LCP of
every neighbour pair), which is equivalent because the answer is unique.
"""
import sys

import numpy as np
import pytest

import gen
from gpu_util import assert_equal_to_oracle, gpu_sort, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 777, 2047, 2048, 2049, 5000, 20000, 100003])
@pytest.mark.parametrize("model", ["random", "bytes", "binary", "markov", "urls"])
def test_models_vs_oracle(model, n):
    note(f"case model={model} n={n}")
    c, o = gen.generate(model, n, 1000 + n)
    p, l = gpu_sort(c, o)
    assert_equal_to_oracle(c, o, p, l, label=f"{model}/{n}")


@pytest.mark.parametrize("n", [5000, 70000])
def test_suffixes_vs_oracle(n):
    note(f"case suffixes n={n}")
    c, o = gen.generate("suffixes", n, 4)
    p, l = gpu_sort(c, o)
    assert_equal_to_oracle(c, o, p, l, label=f"suffixes/{n}")


def test_c0_full_and_ragged():
    for n in (131072, 131072 + 777):
        note(f"case c0 n={n}")
        c, o = gen.workload("c0_random_128k", n)
        p, l = gpu_sort(c, o)
        assert_equal_to_oracle(c, o, p, l, label=f"c0/{n}")


def _adversarial():
    cases = {}
    cases["all_equal"] = [b"abcdefghij"] * 10000
    cases["all_empty"] = [b""] * 5000
    cases["empty_and_zero_bytes"] = [b"", b"\x00", b"\x00\x00", b"", b"\x00\xff", b"\xff", b"\x00"] * 700
    cases["nested_prefixes"] = [b"a" * k for k in range(600, 0, -1)]
    cases["long_identical"] = [bytes(range(256)) * 2] * 3000
    rng = np.random.default_rng(5)
    base = bytes(rng.integers(0, 256, 600, dtype=np.uint8))
    cases["long_common_prefix"] = [base[:512] + bytes([x]) for x in rng.integers(0, 3, 9000)]
    cases["prefix_ladder_bytes"] = [base[:k] for k in rng.integers(0, 520, 12000)]
    # Skyline string (section 6.3): T_i -> T_{i+1} s_i T_{i+1}, all suffixes
    p = 12
    t = b""
    for i in range(p, 0, -1):
        s = bytes([ord("a") + i - 1])
        t = s if i == p else t + s + t
    cases["skyline_suffixes"] = [t[i:] for i in range(len(t))]
    cases["random2_long"] = [bytes(rng.choice([48, 49], rng.integers(1, 200))) for _ in range(20000)]
    cases["duplicates_mixed"] = [bytes(rng.choice([97, 98], rng.integers(0, 20))) for _ in range(30000)]
    return cases


@pytest.mark.parametrize("name", sorted(_adversarial()))
def test_adversarial_vs_oracle(name):
    strings = _adversarial()[name]
    note(f"case adversarial={name} n={len(strings)}")
    c, o = gen.from_list(strings)
    p, l = gpu_sort(c, o)
    assert_equal_to_oracle(c, o, p, l, label=name)


def test_deterministic_repeat():
    c, o = gen.generate("markov", 200000, 9)
    p1, l1 = gpu_sort(c, o)
    p2, l2 = gpu_sort(c, o)
    assert np.array_equal(p1, p2) and np.array_equal(l1, l2)
    assert_equal_to_oracle(c, o, p1, l1, full=False)


def test_empty_input():
    import torch
    import paper_1808_00963_amd as ss
    chars = torch.zeros(0, dtype=torch.uint8, device="cuda")
    offs = torch.zeros(1, dtype=torch.int64, device="cuda")
    p, l = ss.sort(chars, offs)
    assert p.numel() == 0 and l.numel() == 0


def test_bad_offsets_is_an_error_and_context_recovers():
    import torch
    import paper_1808_00963_amd as ss
    ctx = ss.Context()
    c, o = gen.generate("random", 5000, 3)
    bad = o.copy()
    bad[100], bad[101] = bad[101], bad[100]   # not monotone
    from gpu_util import to_device
    cd, od = to_device(c, bad)
    ctx.sort(cd, od)  # asynchronous: the device-side error surfaces at sync
    with pytest.raises(ss.SSError) as e:
        ctx.sync()
    assert e.value.status == ss.SS_LIMIT
    assert ctx.last_error() == ss.SS_LIMIT
    # sticky until cleared, also across later sorts
    p, l = gpu_sort(c, o, ctx=ctx)
    assert ctx.last_error() == ss.SS_LIMIT
    ctx.clear_error()
    assert ctx.last_error() == ss.SS_OK
    p, l = gpu_sort(c, o, ctx=ctx)
    assert_equal_to_oracle(c, o, p, l)


@pytest.mark.parametrize("name,n", [("c1_markov_16m", None), ("c2a_urls_8m", None), ("c2b_suffixes_2m", None)])
def test_full_size_workloads(name, n):
    note(f"case full workload={name}")
    c, o = gen.workload(name, n)
    p, l = gpu_sort(c, o)
    assert_equal_to_oracle(c, o, p, l, full=False, label=name)


@pytest.mark.parametrize("cfg", [dict(max_log_splitters=1, bucket_target=16, base_max=64),
                                 dict(max_log_splitters=3, bucket_target=16, base_max=256),
                                 dict(max_log_splitters=10, bucket_target=16, base_max=300),
                                 dict(max_log_splitters=6, bucket_target=64, base_max=2048),
                                 dict(max_log_splitters=10, bucket_target=2048, base_max=2048)],
                         ids=lambda c: "d{max_log_splitters}_t{bucket_target}_b{base_max}".format(**c))
@pytest.mark.parametrize("model", ["markov", "urls", "bytes", "suffixes"])
def test_tuning_parameters_do_not_change_results(model, cfg):
    import paper_1808_00963_amd as ss
    note(f"case tuning model={model} cfg={cfg}")
    ctx = ss.Context()
    ctx.set_config(**cfg)
    c, o = gen.generate(model, 60000 if model != "suffixes" else 20000, 77)
    p, l = gpu_sort(c, o, ctx=ctx)
    assert_equal_to_oracle(c, o, p, l, label=f"{model}/{cfg}")
