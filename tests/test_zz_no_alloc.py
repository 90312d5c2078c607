"""The entry point that allocates nothing (ss_sort_noalloc, for callers that
cannot allocate) against the context sort (ss_sort_ex) through the C ABI:
two calls in a row on the library's fixed workspace, the second with a
smaller input, each equal element by element to the context sort's output
(the answer is unique, so equal to the oracle's as well)."""
import ctypes
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


def noalloc(cd, od, n, stream):
    import paper_1808_00963_amd as ss
    perm = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    lcp = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    err = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    st = ss.lib().ss_sort_noalloc(ctypes.c_void_p(cd.data_ptr()), ctypes.c_void_p(od.data_ptr()), n,
                                  ctypes.c_void_p(perm.data_ptr()), ctypes.c_void_p(lcp.data_ptr()),
                                  ctypes.c_void_p(err.data_ptr()), ctypes.c_void_p(stream.cuda_stream))
    assert st == ss.SS_OK
    return perm, lcp, err


def context_sort(cd, od, n, stream):
    import paper_1808_00963_amd as ss
    ctx = ss.Context()
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    lcp = torch.empty(n, dtype=torch.int32, device="cuda")
    st = ss.lib().ss_sort_ex(ctx._h, ctypes.c_void_p(cd.data_ptr()), ctypes.c_void_p(od.data_ptr()), n,
                             ctypes.c_void_p(perm.data_ptr()), ctypes.c_void_p(lcp.data_ptr()),
                             ctypes.c_void_p(stream.cuda_stream))
    assert st == ss.SS_OK
    stream.synchronize()
    assert ctx.last_error() == ss.SS_OK
    return to_host(perm), to_host(lcp)


@pytest.mark.parametrize("model", ["markov", "urls", "suffixes"])
def test_noalloc_equals_context_sort_twice(model):
    import paper_1808_00963_amd as ss
    stream = torch.cuda.current_stream()
    sizes = [ss.NOALLOC_MAX_STRINGS, 70001] if model == "markov" else [300000, 4097]
    for k, n in enumerate(sizes):
        note(f"case noalloc model={model} call={k} n={n}")
        c, o = gen.generate(model, n, 900 + k)
        cd, od = to_device(c, o)
        perm, lcp, err = noalloc(cd, od, n, stream)
        stream.synchronize()
        assert int(err.item()) == 0
        p, l = to_host(perm), to_host(lcp)
        ep, el = context_sort(cd, od, n, stream)
        assert np.array_equal(p, ep), f"{model} call {k}: perm differs from ss_sort_ex"
        assert np.array_equal(l, el), f"{model} call {k}: lcp differs from ss_sort_ex"
        if n <= 100000:
            assert_equal_to_oracle(c, o, p, l, label=f"noalloc {model} n={n}")


def test_noalloc_limits_and_device_errors():
    """Beyond the fixed workspace: SS_LIMIT without running anything;
    malformed offsets: the device error word is set, and the next call
    (valid input) starts clean."""
    import paper_1808_00963_amd as ss
    stream = torch.cuda.current_stream()
    c, o = gen.generate("random", 5000, 3)
    cd, od = to_device(c, o)
    st = ss.lib().ss_sort_noalloc(ctypes.c_void_p(cd.data_ptr()), ctypes.c_void_p(od.data_ptr()),
                                  ss.NOALLOC_MAX_STRINGS + 1, None, None, None, ctypes.c_void_p(stream.cuda_stream))
    assert st == ss.SS_LIMIT
    bad = o.copy()
    bad[100], bad[101] = bad[101], bad[100]
    bd, bo = to_device(c, bad)
    _, _, err = noalloc(bd, bo, 5000, stream)
    stream.synchronize()
    assert int(err.item()) != 0
    perm, lcp, err = noalloc(cd, od, 5000, stream)
    stream.synchronize()
    assert int(err.item()) == 0
    assert_equal_to_oracle(c, o, to_host(perm), to_host(lcp), label="after error")
