"""Helpers for GPU parity tests: move seeded inputs to the device, run the
HIP sort through the C ABI binding, compare with the oracle."""
import numpy as np
import pytest
import torch

import oracle

gpu_available = torch.cuda.is_available()
needs_gpu = pytest.mark.skipif(not gpu_available, reason="no GPU")


def to_device(chars, offsets):
    c = torch.from_numpy(np.ascontiguousarray(chars, dtype=np.uint8)).cuda()
    o = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.uint64).view(np.int64)).cuda()
    return c, o


def to_host(t):
    return t.cpu().numpy().view(np.uint32)


def gpu_sort(chars, offsets, ctx=None):
    import paper_1808_00963_amd as ss
    c, o = to_device(chars, offsets)
    if ctx is None:
        perm, lcp = ss.sort(c, o)
    else:
        perm, lcp = ctx.sort(c, o)
    torch.cuda.synchronize()
    return to_host(perm), to_host(lcp)


def assert_equal_to_oracle(chars, offsets, perm, lcp, full=True, label=""):
    """full: element-by-element against the oracle's sort; otherwise the
    oracle's linear-time check (equivalent, since the answer is unique)."""
    n = len(offsets) - 1
    assert perm.shape == (n,) and lcp.shape == (n,)
    if full:
        ep, el = oracle.sort(chars, offsets)
        bad_p = np.nonzero(ep != perm)[0]
        bad_l = np.nonzero(el != lcp)[0]
        assert bad_p.size == 0, f"{label}: perm differs at {bad_p[:10]} (of {bad_p.size})"
        assert bad_l.size == 0, f"{label}: lcp differs at {bad_l[:10]}: got {lcp[bad_l[:10]]} want {el[bad_l[:10]]}"
    else:
        code = oracle.check(chars, offsets, perm, lcp)
        assert code == -1, f"{label}: {oracle.describe_check(code, n)}"
