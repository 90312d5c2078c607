"""ORACLE for the string sorter -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
``paper_1808_00963_amd``) never imports it and shares no code with it.

``sort`` is the definition of the result written out (section 2.1 of the
paper: lexicographic order with a proper prefix smaller, the LCP array H with
its undefined first entry read as 0), with ties broken by original index so
the answer is unique.  ``check`` verifies a claimed answer against the same
definition in linear time; since the answer is unique, passing ``check`` is
equivalent to equality with ``sort``.  ``suffix_array`` and ``h_names`` are
the definitions of the suffix array and of the h-names of prefix doubling
(section 8.2) written out.  See ``ss_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compiles liboracle.so in place with gcc."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=gnu11", "-pthread",
                               os.path.join(_HERE, "ss_oracle.c"), "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def load(path: str | None = None):
    """Loads the oracle library (``path`` overrides, for mutation tests)."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _bind(lib):
    vp, u32 = ctypes.c_void_p, ctypes.c_uint32
    lib.ss_oracle_sort.restype = ctypes.c_int
    lib.ss_oracle_sort.argtypes = [vp, vp, u32, vp, vp]
    lib.ss_oracle_check.restype = ctypes.c_longlong
    lib.ss_oracle_check.argtypes = [vp, vp, u32, vp, vp]
    lib.ss_oracle_lcp.restype = u32
    lib.ss_oracle_lcp.argtypes = [vp, vp, u32, u32]
    lib.ss_oracle_compare.restype = ctypes.c_int
    lib.ss_oracle_compare.argtypes = [vp, vp, u32, u32]
    lib.ss_oracle_sort_mt.restype = ctypes.c_int
    lib.ss_oracle_sort_mt.argtypes = [vp, vp, u32, vp, vp, u32]
    lib.ss_oracle_suffix_array.restype = ctypes.c_int
    lib.ss_oracle_suffix_array.argtypes = [vp, u32, vp]
    lib.ss_oracle_h_names.restype = ctypes.c_int
    lib.ss_oracle_h_names.argtypes = [vp, u32, ctypes.c_uint64, vp]
    return lib


def _prep(chars, offsets):
    chars = np.ascontiguousarray(chars, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    if chars.size == 0:
        chars = np.zeros(1, dtype=np.uint8)
    return chars, offsets


def sort(chars, offsets, lib=None):
    """Returns (perm uint32[n], lcp uint32[n]) for the string set."""
    lib = lib or load()
    chars, offsets = _prep(chars, offsets)
    n = offsets.size - 1
    perm = np.zeros(max(n, 1), dtype=np.uint32)
    lcp = np.zeros(max(n, 1), dtype=np.uint32)
    lib.ss_oracle_sort(chars.ctypes.data, offsets.ctypes.data, n, perm.ctypes.data, lcp.ctypes.data)
    return perm[:n], lcp[:n]


def sort_mt(chars, offsets, threads: int, lib=None):
    """Same result as ``sort``, computed on ``threads`` host threads (chunk
    sorts, pairwise merges, LCPs over disjoint ranges)."""
    lib = lib or load()
    chars, offsets = _prep(chars, offsets)
    n = offsets.size - 1
    perm = np.zeros(max(n, 1), dtype=np.uint32)
    lcp = np.zeros(max(n, 1), dtype=np.uint32)
    if lib.ss_oracle_sort_mt(chars.ctypes.data, offsets.ctypes.data, n, perm.ctypes.data, lcp.ctypes.data,
                             int(threads)) != 0:
        raise MemoryError("ss_oracle_sort_mt")
    return perm[:n], lcp[:n]


def check(chars, offsets, perm, lcp, lib=None) -> int:
    """Returns -1 if (perm, lcp) is the correct output, else an error code
    (see ``ss_oracle_check`` in ss_oracle.c)."""
    lib = lib or load()
    chars, offsets = _prep(chars, offsets)
    n = offsets.size - 1
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    lcp = np.ascontiguousarray(lcp, dtype=np.uint32)
    if perm.size != n or lcp.size != n:
        raise ValueError("perm/lcp size mismatch")
    if n == 0:
        return -1
    return int(lib.ss_oracle_check(chars.ctypes.data, offsets.ctypes.data, n, perm.ctypes.data, lcp.ctypes.data))


def lcp_of(chars, offsets, a: int, b: int, lib=None) -> int:
    """Longest common prefix of strings a and b (character loop)."""
    chars, offsets = _prep(chars, offsets)
    return int((lib or load()).ss_oracle_lcp(chars.ctypes.data, offsets.ctypes.data, a, b))


def compare(chars, offsets, a: int, b: int, lib=None) -> int:
    """-1, 0 or 1: strings a and b compared by (bytes, length, index)."""
    chars, offsets = _prep(chars, offsets)
    return int((lib or load()).ss_oracle_compare(chars.ctypes.data, offsets.ctypes.data, a, b))


def check_sampled(chars, offsets, perm, lcp, positions, lib=None) -> list:
    """Checks a claimed output at the given sorted positions only (for
    outputs too large for a full oracle run): each sampled pair
    (perm[k-1], perm[k]) must be strictly increasing in (string, index)
    order and lcp[k] must equal their common prefix; lcp[0] must be 0.
    Returns descriptions of the failures (empty = all sampled positions
    agree with the definition)."""
    lib = lib or load()
    chars, offsets = _prep(chars, offsets)
    n = offsets.size - 1
    fails = []
    for k in positions:
        k = int(k)
        if k == 0:
            if n and int(lcp[0]) != 0:
                fails.append("lcp[0] != 0")
            continue
        a, b = int(perm[k - 1]), int(perm[k])
        if a >= n or b >= n:
            fails.append(f"perm entry out of range at {k}")
            continue
        if int(lib.ss_oracle_compare(chars.ctypes.data, offsets.ctypes.data, a, b)) >= 0:
            fails.append(f"order violated at sorted position {k}")
        want = int(lib.ss_oracle_lcp(chars.ctypes.data, offsets.ctypes.data, a, b))
        if int(lcp[k]) != want:
            fails.append(f"lcp at {k}: got {int(lcp[k])}, want {want}")
    return fails


def _text(text):
    t = np.ascontiguousarray(np.frombuffer(text, dtype=np.uint8) if isinstance(text, (bytes, bytearray))
                             else text, dtype=np.uint8)
    return t, (t if t.size else np.zeros(1, dtype=np.uint8))


def suffix_array(text, lib=None):
    """Suffix array (uint32[n]) of a byte text, no sentinel appended."""
    lib = lib or load()
    t, buf = _text(text)
    sa = np.zeros(max(t.size, 1), dtype=np.uint32)
    lib.ss_oracle_suffix_array(buf.ctypes.data, t.size, sa.ctypes.data)
    return sa[:t.size]


def h_names(text, h: int, lib=None):
    """Lexicographic h-names (smallest rank in h-order) of all suffixes."""
    lib = lib or load()
    t, buf = _text(text)
    names = np.zeros(max(t.size, 1), dtype=np.uint32)
    if lib.ss_oracle_h_names(buf.ctypes.data, t.size, h, names.ctypes.data) != 0:
        raise MemoryError("ss_oracle_h_names")
    return names[:t.size]


def describe_check(code: int, n: int) -> str:
    if code == -1:
        return "ok"
    if code < n:
        return f"wrong lcp at sorted position {code}"
    if code < 2 * n:
        return f"order violated at sorted position {code - n}"
    if code < 3 * n:
        return f"not a permutation (entry {code - 2 * n})"
    return "lcp[0] != 0"
