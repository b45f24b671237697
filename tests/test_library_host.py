"""CPU checks of libsgmdi.so: it loads, exports every symbol of
include/sgmdi.h, and its host-side integer layer and rule tables agree
with the oracle (bit-exact for integers)."""
import os
import re

import numpy as np
import pytest

from oracle import counts as OC
from paper_2210_14313_amd import native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    return native.lib()


def test_library_exports_every_declared_symbol(L):
    hdr = open(os.path.join(ROOT, "include", "sgmdi.h")).read()
    declared = set(re.findall(r"^(?:sg_status|const char \*)\s*(sg_\w+)\s*\(", hdr, flags=re.M))
    assert declared == set(native.EXPORTS), declared ^ set(native.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_status_strings(L):
    for s in range(7):
        assert L.sg_status_string(s)


CASES = [(d, q, r) for r in ("tr", "cc", "gl", "gl_paper", "gp")
         for d, q in [(1, 1), (1, 6), (2, 4), (2, 9), (3, 7), (5, 9), (7, 12), (10, 14), (12, 12)]]


@pytest.mark.parametrize("d,q,rule", CASES)
def test_counts_bit_exact_small(d, q, rule):
    got = native.counts(d, q, rule)
    ref = OC.counts_by_generating_function(d, q, rule)
    assert got == (ref["n_multi"], ref["n_points_rep"], ref["n_points_unique"])
    en = OC.counts_by_enumeration(d, q, rule) if d <= 7 and q - d <= 6 else None
    if en:
        assert got[:2] == (en["n_multi"], en["n_points_rep"])


@pytest.mark.parametrize("d,q,rule", [(100, 105, "cc"), (1000, 1003, "gl"), (1000, 1003, "tr"),
                                      (200, 205, "cc"), (256, 262, "cc"), (256, 262, "gl"),
                                      (10, 14, "cc"), (5, 18, "gl_paper"), (10, 21, "gl_paper")])
def test_counts_bit_exact_large(d, q, rule):
    got = native.counts(d, q, rule)
    ref = OC.counts_by_generating_function(d, q, rule)
    assert got == (ref["n_multi"], ref["n_points_rep"], ref["n_points_unique"])


def test_counts_overflow_is_reported():
    with pytest.raises(native.SgError) as e:
        native.counts(10 ** 6, 10 ** 6 + 6, "cc")
    assert e.value.status == 3
    with pytest.raises(native.SgError) as e:
        native.counts(0, 3, "cc")
    assert e.value.status == 1
    with pytest.raises(native.SgError) as e:
        native.counts(3, 2, "cc")
    assert e.value.status == 1
    # an unknown rule id
    assert native.lib().sg_counts(3, 5, 6, None, None, None) == 1


@pytest.mark.parametrize("d,q", [(1, 4), (2, 5), (3, 7), (5, 9), (6, 8), (9, 11)])
def test_unrank_matches_oracle_enumeration(orc, d, q):
    total, coords, levels, nnz = orc.enumerate_window(d, q)
    assert total == native.counts(d, q, "cc")[0]
    for r in range(total):
        got = native.unrank(d, q, r)
        ref = [(int(coords[r, k]), int(levels[r, k])) for k in range(nnz[r])]
        assert got == ref, (r, got, ref)
    with pytest.raises(native.SgError):
        native.unrank(d, q, total)


def test_unrank_large_window_spot_checks(orc):
    # d = 1000, K = 3: compare ranks in every excess class against a direct
    # walk of the oracle's order on a smaller prefix, and invariants elsewhere
    d, q = 1000, 1003
    n = native.counts(d, q, "cc")[0]
    rng = np.random.default_rng(0)
    prev = None
    for r in sorted(set([0, 1, 2, n - 1, n - 2] + list(rng.integers(0, n, 200)))):
        mi = native.unrank(d, q, int(r))
        assert all(0 <= c < d for c, _ in mi) and all(l >= 2 for _, l in mi)
        assert [c for c, _ in mi] == sorted(c for c, _ in mi)
        e = sum(l - 1 for _, l in mi)
        assert 0 <= e <= 3
        key = (e, tuple(-x for x in _dense(mi, d)))
        if prev is not None:
            assert key > prev
        prev = key
    total, coords, levels, nnz = orc.enumerate_window(d, q, 0, 5000)
    for r in range(5000):
        ref = [(int(coords[r, k]), int(levels[r, k])) for k in range(nnz[r])]
        assert native.unrank(d, q, r) == ref


def _dense(mi, d):
    v = [1] * min(d, 64)
    out = dict(mi)
    return tuple(out.get(i, 1) for i in range(d))


@pytest.mark.parametrize("d,q", [(1, 1), (3, 6), (10, 14), (100, 105), (1000, 1003), (256, 262)])
def test_coefficients_match_oracle(d, q):
    for e in range(0, q - d + 1):
        assert native.coefficient(d, q, e) == OC.coefficient(d, q, e) * (e in OC.window(d, q))


@pytest.mark.parametrize("rule", ["tr", "cc", "gl", "gl_paper", "gp"])
def test_rule_tables_match_oracle(orc, rule):
    for level in range(1, 9):
        x, w = native.rule_table(rule, level)
        xo, wo = orc.rule(rule, level)
        np.testing.assert_allclose(x, xo, rtol=0, atol=2e-16)
        np.testing.assert_allclose(w, wo, rtol=4e-16, atol=1e-18)


@pytest.mark.parametrize("d,q,rule", [(3, 8, "gl"), (4, 7, "cc"), (2, 5, "tr"), (1, 6, "gl_paper"), (5, 5, "cc")])
def test_point_path_work_count_by_brute_force(d, q, rule):
    # the benchmark's flop-slot count of the point-by-point sum: points of
    # the window of (2.6) and the number of active coordinates over them
    import itertools
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    K = q - d
    n = [len(native.rule_table(rule, l)[0]) for l in range(1, K + 2)]
    P = S = 0
    for l in itertools.product(range(1, K + 2), repeat=d):
        if not (max(d, q - d + 1) <= sum(l) <= q):
            continue
        pp = int(np.prod([n[x - 1] for x in l]))
        P += pp
        S += pp * sum(1 for x in l if x >= 2)
    assert bench.points_flop_slots(d, q, rule) == (P, 9 * P + 2 * S)
    assert P == OC.counts_by_generating_function(d, q, rule)["n_points_rep"]


def test_gauss_patterson_counts_match_the_paper():
    # distinct points of the Gauss-Patterson sparse grids printed in
    # Tables 4.1, 4.3 and 4.5 (accuracy level q -> excess q - 1)
    import json
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                    "paper_gp_node_counts.json")))
    for row in g["rows"]:
        d, q = row["d"], row["q"]
        assert native.counts(d, d + q - 1, "gp")[2] == row["unique_points"], row


def test_peaks_library_exports_every_declared_symbol():
    from paper_2210_14313_amd import peaks
    hdr = open(os.path.join(ROOT, "include", "sgpeaks.h")).read()
    declared = set(re.findall(r"^(?:int32_t|const char \*)\s*(sgp_\w+)\s*\(", hdr, flags=re.M))
    assert declared == set(peaks.EXPORTS), declared ^ set(peaks.EXPORTS)
    L = peaks.lib()
    for name in declared:
        assert hasattr(L, name), name
    names = [L.sgp_op_name(i).decode() for i in range(len(peaks.OPS))]
    assert names == list(peaks.OPS), names
    assert L.sgp_op_name(len(peaks.OPS)) == b""


def test_peaks_rejects_bad_arguments_before_launch():
    import ctypes
    from paper_2210_14313_amd import peaks
    L = peaks.lib()
    sink = ctypes.c_void_p(16)     # never dereferenced: every call below is rejected first
    assert L.sgp_launch(-1, 1, 1, sink, None, None, None) == 1
    assert L.sgp_launch(len(peaks.OPS), 1, 1, sink, None, None, None) == 1
    assert L.sgp_launch(0, 0, 1, sink, None, None, None) == 1
    assert L.sgp_launch(0, 1, 0, sink, None, None, None) == 1
    assert L.sgp_launch(0, 1, 1, None, None, None, None) == 1
