"""The oracle pinned to results fixed by the paper and by mathematics (CPU)."""
import os
import subprocess

import numpy as np
import pytest

import gen
import oracle
import pins


@pytest.fixture(scope="module")
def lib():
    oracle.build(force=False)
    return oracle.load()


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(lib, pin):
    assert pin(lib) == []


def test_check_accepts_oracle_and_rejects_planted_errors(lib):
    c, o = gen.generate("bytes", 3000, 5)
    p, l = oracle.sort(c, o)
    n = len(p)
    assert oracle.check(c, o, p, l) == -1
    # a wrong LCP entry
    l2 = l.copy(); l2[10] += 1
    assert oracle.check(c, o, p, l2) == 10
    # two neighbours swapped
    p2 = p.copy(); p2[20], p2[21] = p2[21], p2[20]
    assert n <= oracle.check(c, o, p2, l) < 2 * n
    # not a permutation
    p3 = p.copy(); p3[5] = p3[6]
    assert 2 * n <= oracle.check(c, o, p3, l) < 3 * n
    # nonzero first entry
    l3 = l.copy(); l3[0] = 1
    assert oracle.check(c, o, p, l3) == 3 * n


def test_check_equals_sort_on_workload_slices(lib):
    for name in gen.WORKLOADS:
        c, o = gen.workload(name, 5000)
        p, l = oracle.sort(c, o)
        assert oracle.check(c, o, p, l) == -1, name


def test_empty_and_single(lib):
    p, l = oracle.sort(np.zeros(0, np.uint8), np.zeros(1, np.uint64))
    assert p.size == 0 and l.size == 0
    c, o = gen.from_list([b"x"])
    p, l = oracle.sort(c, o)
    assert p.tolist() == [0] and l.tolist() == [0]


# Plausible mistakes planted in copies of the oracle source: every one must
# be caught by at least one pin.
MUTATIONS = {
    "signed_bytes": ("int c = m ? memcmp(sa, sb, (size_t)m) : 0;",
                     "int c = 0; for (uint64_t q = 0; q < m && !c; ++q) c = (signed char)sa[q] - (signed char)sb[q];"),
    "longer_prefix_first": ("if (la != lb) return la < lb ? -1 : 1;", "if (la != lb) return la > lb ? -1 : 1;"),
    "ties_reversed": ("if (a != b) return a < b ? -1 : 1;", "if (a != b) return a > b ? -1 : 1;"),
    "dropped_last_char": ("int c = m ? memcmp(sa, sb, (size_t)m) : 0;", "int c = m > 1 ? memcmp(sa, sb, (size_t)(m - 1)) : 0;"),
    "lcp_without_perm": ("lcp[k] = lcp_brute(&S, perm[k - 1], perm[k]);", "lcp[k] = lcp_brute(&S, k - 1, k);"),
    "lcp_off_by_one": ("while (k < m && sa[k] == sb[k]) ++k;", "while (k < m && sa[k] == sb[k]) ++k; if (k < m) ++k;"),
    "lcp0_bottom": ("if (n) lcp[0] = 0;", "if (n) lcp[0] = n > 1 ? lcp_brute(&S, perm[0], perm[1]) : 0;"),
    "suffix_prefix_last": ("if (la != lb) return la < lb ? -1 : 1; /* proper prefix is smaller */",
                           "if (la != lb) return la > lb ? -1 : 1;"),
    "h_names_by_position": ("names[order[k]] = first;", "names[order[k]] = k;"),
    "h_truncation_dropped": ("if (la > S->h) la = S->h;", ""),
    "mt_merge_drops_tail": ("while (b < j->hi) j->dst[o++] = j->src[b++];", ""),
    "mt_merge_prefers_right": ("cmp_idx(j->S, j->src[a], j->src[b]) < 0 ? j->src[a++] : j->src[b++];",
                               "cmp_idx(j->S, j->src[a], j->src[b]) > 0 ? j->src[a++] : j->src[b++];"),
    "mt_lcp_without_perm": ("j->lcp[k] = k ? lcp_brute(j->S, j->src[k - 1], j->src[k]) : 0;",
                            "j->lcp[k] = k ? lcp_brute(j->S, k - 1, k) : 0;"),
    "compare_negated": ("    return cmp_idx(&S, a, b);\n}", "    return -cmp_idx(&S, a, b);\n}"),
    "pair_lcp_off_by_one": ("    return lcp_brute(&S, a, b);\n}", "    return lcp_brute(&S, a, b) + 1;\n}"),
    "suffix_one_char_short": ("int c = m ? memcmp(S->text + a, S->text + b, (size_t)m) : 0;",
                              "int c = m > 1 ? memcmp(S->text + a, S->text + b, (size_t)(m - 1)) : 0;"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutated_oracle_is_caught(tmp_path, name):
    """The pins run against the mutated build in a child process: a mutation
    that makes the oracle crash (e.g. a merge that leaves indices
    uninitialised) counts as caught, like a failed pin."""
    import sys
    src = open(os.path.join(os.path.dirname(oracle.__file__), "ss_oracle.c")).read()
    old, new = MUTATIONS[name]
    assert old in src, f"mutation anchor missing: {old}"
    mutated = tmp_path / "m.c"
    mutated.write_text(src.replace(old, new))
    so = tmp_path / "libm.so"
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-std=gnu11", "-pthread", str(mutated), "-o", str(so)])
    here = os.path.dirname(os.path.abspath(__file__))
    code = ("import sys; sys.path[:0] = [%r, %r]; import oracle, pins; "
            "f = pins.run_all(oracle.load(%r)); print(len(f)); sys.exit(0 if f else 3)"
            % (here, os.path.dirname(here), str(so)))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode != 3, f"mutation {name} was not caught by any pin"
    assert r.returncode != 0 or int(r.stdout.strip().splitlines()[-1]) > 0
