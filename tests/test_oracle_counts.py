"""Pins for the oracle's integer layer (Section 2.1: N_{d,s}, the window of
(2.6), n_d^q, the union (2.4)) and its canonical enumeration order."""
import json
import os
from itertools import product
from math import comb

import pytest

from oracle import counts as C

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_paper_example_N_2_4():
    # Section 2.1: N_{2,4} = {[1,3], [2,2], [3,1]}
    top = [l for l in C.enumerate_window(2, 4) if sum(l) == 4]
    assert sorted(top) == sorted([(1, 3), (2, 2), (3, 1)])


def _brute_window(d, q):
    return [l for l in product(range(1, q + 1), repeat=d) if q - d + 1 <= sum(l) <= q]


@pytest.mark.parametrize("d,q", [(1, 1), (1, 4), (2, 2), (2, 5), (3, 3), (3, 7), (4, 8), (5, 7)])
def test_enumeration_is_the_window_in_canonical_order(d, q):
    got = C.enumerate_window(d, q)
    brute = _brute_window(d, q)
    assert sorted(got) == sorted(brute)
    key = [(sum(l), tuple(-x for x in l)) for l in got]
    assert key == sorted(key)          # excess ascending, then decreasing lex
    assert len(set(got)) == len(got)


@pytest.mark.parametrize("rule", ["tr", "cc", "gl", "gl_paper", "gp"])
@pytest.mark.parametrize("d,q", [(1, 1), (1, 5), (2, 4), (2, 7), (3, 6), (3, 8), (4, 7), (5, 9), (6, 8)])
def test_generating_function_matches_enumeration(rule, d, q):
    gf = C.counts_by_generating_function(d, q, rule)
    en = C.counts_by_enumeration(d, q, rule)
    assert gf["n_multi"] == en["n_multi"]
    assert gf["n_points_rep"] == en["n_points_rep"]
    assert gf["n_points_unique"] == C.unique_points_by_enumeration(d, q, rule)


@pytest.mark.parametrize("d,K", [(2, 1), (5, 3), (10, 4), (100, 5), (1000, 3)])
def test_multi_index_identities(d, K):
    q = d + K
    got = C.counts_by_generating_function(d, q, "cc")["n_multi"]
    # K <= d-1: the window holds every l with |l| - d <= K, i.e. C(d+K, K) of them
    assert got == comb(d + K, K)
    # the combination coefficients weight the window to total 1 (Q(1) = 1)
    s = sum(C.coefficient(d, q, e) * comb(d - 1 + e, e) for e in C.window(d, q))
    assert s == 1


def test_paper_table_5_6_node_counts():
    g = json.load(open(os.path.join(GOLDEN, "paper_node_counts.json")))
    for row in g["rows"]:
        d, N = row["d"], row["N"]
        assert C.unique_points_by_generating_function(d, d + N - 1, g["rule"]) == row["unique_points"], row
    for row in g["rows"][:3]:
        d, N = row["d"], row["N"]
        assert C.unique_points_by_enumeration(d, d + N - 1, g["rule"]) == row["unique_points"]


def test_paper_gauss_patterson_node_counts():
    # Tables 4.1, 4.3, 4.5: the Gauss-Patterson level map and its nesting
    g = json.load(open(os.path.join(GOLDEN, "paper_gp_node_counts.json")))
    for row in g["rows"]:
        d, q = row["d"], row["q"]
        assert C.unique_points_by_generating_function(d, d + q - 1, g["rule"]) == row["unique_points"], row
        if d <= 3:
            assert C.unique_points_by_enumeration(d, d + q - 1, g["rule"]) == row["unique_points"], row


def test_small_textbook_counts():
    # d=1: the rule reduces to the single level-q rule
    assert C.counts_by_generating_function(1, 4, "cc") == dict(n_multi=1, n_points_rep=9, n_points_unique=9)
    # d=2, q=4 (K=2), Clenshaw-Curtis: the classic 13-point grid
    g = C.counts_by_generating_function(2, 4, "cc")
    assert g["n_multi"] == 5 and g["n_points_rep"] == 25 and g["n_points_unique"] == 13


@pytest.mark.parametrize("d,q", [(1, 3), (2, 5), (3, 6), (4, 8), (6, 9), (7, 7)])
def test_c_enumeration_matches_python(orc, d, q):
    total, coords, levels, nnz = orc.enumerate_window(d, q)
    ref = C.enumerate_window(d, q)
    assert total == len(ref)
    for r, l in enumerate(ref):
        sparse = [(i, li) for i, li in enumerate(l) if li >= 2]
        assert nnz[r] == len(sparse)
        assert [(int(coords[r, k]), int(levels[r, k])) for k in range(nnz[r])] == sparse
