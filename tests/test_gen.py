"""Seeded generators: determinism, thread independence, model shapes (CPU)."""
import hashlib
import os
import subprocess
import sys

import numpy as np

import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _digest(c, o):
    return hashlib.sha256(o.tobytes() + c.tobytes()).hexdigest()[:16]


def test_deterministic_and_thread_independent():
    c, o = gen.generate("markov", 20000, 2)
    c2, o2 = gen.generate("markov", 20000, 2)
    assert _digest(c, o) == _digest(c2, o2)
    code = ("import sys; sys.path.insert(0, %r); import gen, hashlib; c, o = gen.generate('markov', 20000, 2); "
            "print(hashlib.sha256(o.tobytes() + c.tobytes()).hexdigest()[:16])" % ROOT)
    out = subprocess.check_output([sys.executable, "-c", code], env=dict(os.environ, OMP_NUM_THREADS="1"))
    assert out.decode().strip() == _digest(c, o)


def test_model_shapes():
    c, o = gen.generate("random", 50000, 1)
    L = np.diff(o)
    assert L.min() >= 1 and L.max() <= 32 and c.min() >= ord("a") and c.max() <= ord("z")
    c, o = gen.generate("markov", 50000, 2)
    L = np.diff(o)
    assert L.min() >= 1 and L.max() <= 512 and 40 <= np.median(L) <= 41
    sym = set(b"-0123456789ABCDEFGHIJKLMNOPQRSTUVWXYZ_abcdefghijklmnopqrstuvwxyz")
    assert set(np.unique(c).tolist()) <= sym
    c, o = gen.generate("urls", 20000, 3)
    s = gen.to_list(c, o)
    assert all(x.startswith(b"http://") or x.startswith(b"https://") for x in s)
    assert all(1 <= x.count(b"/") - 2 <= 6 for x in s)
    c, o = gen.generate("suffixes", 8192, 4)
    s = gen.to_list(c, o)
    assert len(s[0]) == 512 and s[-1] == s[-2][1:] and len(s[-1]) == 1
    assert set(np.unique(c).tolist()) <= set(b"ACGT")


def test_batch_sets_shape():
    c, o, b = gen.batch_sets(num_sets=16, seed=5, scale=0.01)
    assert b[0] == 0 and b[-1] == len(o) - 1 and np.all(np.diff(b.astype(np.int64)) >= 2)
    assert int(o[-1]) == len(c)
