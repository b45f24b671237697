"""Exact integer counts of the Smolyak window -- TEST INFRASTRUCTURE ONLY.

Section 2.1: the rule (2.6) sums over multi-indices l >= 1 with
q-d+1 <= |l| <= q; the point count with repetition is
n_d^q = sum over that window of n_{l_1} ... n_{l_d}; the sparse grid (2.4)
is the union of the tensor grids.  Two independent evaluations are given:
plain enumeration (small cases) and generating functions (any size), both in
Python integers, so they are exact.
"""
from __future__ import annotations

from fractions import Fraction
from itertools import product
from math import comb
from typing import Dict, List, Tuple


def n_level(rule: str, level: int) -> int:
    """Points of the level-l 1-D rule (Section 2.2; level 1 = one midpoint)."""
    if level < 1:
        raise ValueError(level)
    if rule in ("tr", "cc"):
        return 1 if level == 1 else 2 ** (level - 1) + 1
    if rule == "gl":
        return 2 * level - 1
    if rule == "gl_paper":
        return level
    if rule == "gp":
        # Gauss-Patterson, level-to-points map of Section 5.4 (q = 1..10)
        if level > 10:
            raise ValueError(level)
        return (1, 3, 3, 7, 7, 7, 15, 15, 15, 15)[level - 1]
    raise ValueError(rule)


def window(d: int, q: int) -> range:
    """Excess values e = |l| - d of the window q-d+1 <= |l| <= q in (2.6)."""
    K = q - d
    return range(max(0, K - d + 1), K + 1)


def coefficient(d: int, q: int, e: int) -> int:
    """(-1)^(q-|l|) C(d-1, q-|l|) of (2.6) for |l| = d + e."""
    K = q - d
    return (-1) ** (K - e) * comb(d - 1, K - e)


# ---------------------------------------------------------------- enumeration
def compositions(e: int, d: int):
    """All l in N^d (l_i >= 1) with |l| = d + e, decreasing lexicographic order."""
    if d == 1:
        yield (e + 1,)
        return
    for k in range(e, -1, -1):
        for rest in compositions(e - k, d - 1):
            yield (k + 1,) + rest


def enumerate_window(d: int, q: int) -> List[Tuple[int, ...]]:
    """Every multi-index of the window, excess ascending then decreasing lex."""
    out = []
    for e in window(d, q):
        out.extend(compositions(e, d))
    return out


def counts_by_enumeration(d: int, q: int, rule: str) -> Dict[str, int]:
    """Multi-index count and n_d^q by walking the window (small cases only)."""
    n_multi = 0
    n_rep = 0
    for l in enumerate_window(d, q):
        n_multi += 1
        p = 1
        for li in l:
            p *= n_level(rule, li)
        n_rep += p
    return dict(n_multi=n_multi, n_points_rep=n_rep)


def _node_ids(rule: str, level: int) -> List[object]:
    """Identity of each node of a level, equal across levels iff the nodes coincide.

    Nested rules (trapezoidal, Clenshaw-Curtis) place node j of an n-point
    level at a position fixed by the fraction j/(n-1), so that fraction is the
    identity (Gauss-Patterson: (j+1)/(n+1)).  Gauss-Legendre levels share only the centre (the zero of the odd
    Legendre polynomials); any other node is identified by (level, index).
    """
    n = n_level(rule, level)
    if n == 1:
        return [Fraction(1, 2)] if rule in ("tr", "cc", "gp") else ["centre"]
    if rule in ("tr", "cc"):
        return [Fraction(j, n - 1) for j in range(n)]
    if rule == "gp":
        # each Patterson extension interlaces its new nodes with the old
        # ones, so node j of an n-point level is node 2j+1 of the next:
        # (j+1)/(n+1) identifies it on every finer level
        return [Fraction(j + 1, n + 1) for j in range(n)]
    ids: List[object] = []
    for j in range(n):
        if n % 2 == 1 and j == n // 2:
            ids.append("centre")
        else:
            ids.append((level, j))
    return ids


def unique_points_by_enumeration(d: int, q: int, rule: str) -> int:
    """Size of the union of all tensor grids of the window (small cases only)."""
    pts = set()
    for l in enumerate_window(d, q):
        for p in product(*[_node_ids(rule, li) for li in l]):
            pts.add(p)
    return len(pts)


# ----------------------------------------------------------- generating funcs
def _poly_pow_trunc(coef: List[int], power: int, K: int) -> List[int]:
    """coef(z)^power truncated after z^K, exact integers (square and multiply)."""
    def mul(a, b):
        r = [0] * (K + 1)
        for i, ai in enumerate(a):
            if ai == 0:
                continue
            for j in range(0, K + 1 - i):
                r[i + j] += ai * b[j]
        return r
    result = [1] + [0] * K
    base = (list(coef) + [0] * (K + 1))[:K + 1]
    while power:
        if power & 1:
            result = mul(result, base)
        base = mul(base, base)
        power >>= 1
    return result


def counts_by_generating_function(d: int, q: int, rule: str) -> Dict[str, int]:
    """Counts from generating functions.

    Multi-indices of excess e: C(d-1+e, e).  Points with repetition:
    [z^e] N(z)^d with N(z) = sum_l n_l z^(l-1).  Unique points: see
    ``unique_points_by_generating_function``.
    """
    K = q - d
    N = [n_level(rule, l + 1) for l in range(K + 1)]
    NP = _poly_pow_trunc(N, d, K)
    n_multi = sum(comb(d - 1 + e, e) for e in window(d, q))
    n_rep = sum(NP[e] for e in window(d, q))
    return dict(n_multi=n_multi, n_points_rep=n_rep,
                n_points_unique=unique_points_by_generating_function(d, q, rule))


def unique_points_by_generating_function(d: int, q: int, rule: str) -> int:
    """Number of distinct points of the sparse grid.

    Nested rules (trapezoidal, Clenshaw-Curtis, Gauss-Patterson): a point
    is in the grid iff the levels at which its coordinates first appear sum
    to at most q, so the count is
    sum_{e<=K} [z^e] M(z)^d with M(z) = sum_l (n_l - n_{l-1}) z^(l-1).

    Gauss-Legendre: a coordinate either sits at the centre (present at every
    level with an odd point count) or at a node owned by one level.  With c
    centre coordinates and non-centre excess E, the point is in the grid iff
    some window multi-index reaches it; see the inline conditions.
    """
    K = q - d
    if rule in ("tr", "cc", "gp"):
        M = [n_level(rule, 1)] + [n_level(rule, l) - n_level(rule, l - 1) for l in range(2, K + 2)]
        MP = _poly_pow_trunc(M, d, K)
        return sum(MP[: K + 1])
    # Gauss-Legendre: non-centre nodes per level
    nc = [0] + [n_level(rule, l) - (n_level(rule, l) % 2) for l in range(2, K + 2)]
    total = 0
    for c in range(0, d + 1):
        G = _poly_pow_trunc(nc, d - c, K)      # z^E <-> non-centre excess E
        for E in range(0, K + 1):
            if G[E] == 0:
                continue
            if c == 0:
                ok = K - d + 1 <= E <= K
            elif rule == "gl":
                ok = E <= K                       # centre levels free: any |l| >= E + d
            else:
                # paper count n_l = l: the centre is only in odd levels, so the
                # reachable level sums are E + d + 2j, j >= 0
                lo, hi = q - d + 1, q
                s = E + d
                ok = s <= hi and any(lo <= s + 2 * j <= hi for j in range(0, (hi - s) // 2 + 1))
            if ok:
                total += comb(d, c) * G[E]
    return total


def effective_points(problems) -> int:
    """Sum of n_d^q over a list of problems (the effective-points numerator)."""
    return sum(counts_by_generating_function(p.d, p.q, p.rule)["n_points_rep"] for p in problems)
