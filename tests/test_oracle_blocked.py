"""Pins for the oracle's block (tensor-product) variant of the sparse grid
(the reading of Algorithm 3.3 with step m > 1, (3.8)-(3.11)).

The oracle forms the product of block values; these tests check it against
the rule written out literally (every block's sparse grid as a list of
weighted points, their tensor product as a list of d-dimensional points,
the integrand evaluated at each, with rules built by numpy), against the
plain rule when one block covers every coordinate, against polynomial
exactness with a separate budget per block, and against the growth of the
paper's printed errors with the number of blocks (Table 5.2, first order).
"""
from itertools import product
from math import comb

import mpmath as mp
import numpy as np
import pytest

from oracle import blocked as B
from oracle import reference as R
from paper_2210_14313_amd import workloads as W
from test_oracle_values import _f, _level_needed, _numpy_rule


def _sparse_grid_points(db, K, rule):
    """The block's sparse grid (2.6)-(2.7) as weighted points with
    repetition: coefficient times tensor weights, over the window."""
    q = db + K
    pts, wts = [], []
    for l in product(range(1, q + 1), repeat=db):
        s = sum(l)
        if not (q - db + 1 <= s <= q):
            continue
        rules = [_numpy_rule(rule, li) for li in l]
        coef = (-1) ** (q - s) * comb(db - 1, q - s)
        for combo in product(*[range(len(r[0])) for r in rules]):
            pts.append([rules[i][0][j] for i, j in enumerate(combo)])
            wts.append(coef * np.prod([rules[i][1][j] for i, j in enumerate(combo)]))
    return np.array(pts), np.array(wts)


def brute_blocked(d, q, rule, family, params, m):
    """Tensor product of the block grids, evaluated point by point."""
    K = q - d
    grids = [_sparse_grid_points(ln, K, rule) for _, ln in B.blocks(d, m)]
    total = []
    for combo in product(*[range(len(g[1])) for g in grids]):
        x = np.concatenate([grids[b][0][j] for b, j in enumerate(combo)])
        w = np.prod([grids[b][1][j] for b, j in enumerate(combo)])
        total.append(w * _f(family, params, x[None, :])[0])
    return float(mp.fsum(total))


CASES = [(3, 2, "cc", 1), (4, 2, "gl", 2), (4, 3, "gl_paper", 2), (5, 1, "cc", 2), (5, 2, "tr", 3), (3, 4, "cc", 3)]


@pytest.mark.parametrize("d,K,rule,m", CASES)
@pytest.mark.parametrize("family", ["exp_sum", "oscillatory", "product_peak", "gaussian", "oscillatory_quadratic",
                                    "oscillatory_quadratic_linear"])
def test_blocked_equals_the_literal_tensor_product(orc, d, K, rule, m, family):
    rng = np.random.default_rng(100 * d + 10 * K + m)
    params = W.draw_params(rng, family, d)
    ref = brute_blocked(d, d + K, rule, family, params, m)
    for method in ("points", "factorised"):
        got = B.smolyak_blocked(d, d + K, rule, family, params, m, method)
        osc = family in ("oscillatory", "oscillatory_quadratic", "oscillatory_quadratic_linear")
        assert abs(got - ref) <= 1e-13 * max(abs(ref), 1e-3 if osc else 0.0), (method, got, ref)


@pytest.mark.parametrize("family", ["exp_sum", "oscillatory", "product_peak"])
def test_one_block_is_the_plain_rule(orc, family):
    rng = np.random.default_rng(7)
    d, K = 9, 4
    params = W.draw_params(rng, family, d)
    plain = orc.smolyak_points(d, d + K, "cc", family, params)["q"]
    for m in (d, d + 5):
        got = B.smolyak_blocked(d, d + K, "cc", family, params, m, "points")
        assert abs(got - plain) <= 1e-14 * max(abs(plain), 1.0)


def test_single_coordinate_blocks_are_the_full_tensor_rule(orc):
    # m = 1: each coordinate gets the level-(K+1) rule, so the rule is the
    # full tensor product U^{K+1} x ... x U^{K+1}
    rng = np.random.default_rng(8)
    d, K = 3, 3
    c = W.draw_params(rng, "exp_sum", d)
    x, w = _numpy_rule("gl", K + 1)
    X = np.stack(np.meshgrid(*([x] * d), indexing="ij"), -1).reshape(-1, d)
    Wt = np.prod(np.stack(np.meshgrid(*([w] * d), indexing="ij"), -1).reshape(-1, d), axis=-1)
    ref = float(mp.fsum(Wt * np.exp(X @ c)))
    got = B.smolyak_blocked(d, d + K, "gl", "exp_sum", c, 1, "points")
    assert abs(got - ref) <= 1e-14 * ref


@pytest.mark.parametrize("rule", ["cc", "gl"])
def test_polynomial_exactness_with_a_budget_per_block(orc, rule):
    # prod (x_i - 1/2)^alpha_i is integrated exactly iff every block's
    # levels that integrate its factors exactly fit into that block's
    # budget K; the plain rule, with one shared budget, is not exact on
    # the same monomial
    d, m, K = 4, 2, 2
    ones = [a for a in range(0, 12, 2) if _level_needed(rule, a) == 1][-1]
    alpha = np.array([ones, ones, ones, ones])       # each block needs 2 = K
    exact = float(np.prod([((0.5) ** (a + 1) - (-0.5) ** (a + 1)) / (a + 1) for a in alpha]))
    prm = np.concatenate([alpha, [0.5]])
    got = B.smolyak_blocked(d, d + K, rule, "monomial", prm, m, "points")
    assert abs(got - exact) <= 1e-15 * abs(exact)
    plain = orc.smolyak_points(d, d + K, rule, "monomial", prm)["q"]
    assert abs(plain - exact) > 1e-10 * abs(exact)
    # one block over budget: not exact
    two = [a for a in range(0, 12, 2) if _level_needed(rule, a) == 2][-1]
    alpha2 = np.array([two, ones, 0, 0])                 # first block needs 3 > K
    exact2 = float(np.prod([((0.5) ** (a + 1) - (-0.5) ** (a + 1)) / (a + 1) for a in alpha2]))
    got2 = B.smolyak_blocked(d, d + K, rule, "monomial", np.concatenate([alpha2, [0.5]]), m, "points")
    assert abs(got2 - exact2) > 1e-10 * abs(exact2)


def test_paper_table_5_2_errors_grow_with_the_number_of_blocks(orc):
    # Table 5.2, r = 4: Gauss-Legendre with n_l = l, accuracy level 10
    # (q = d + 9), step m = 10, integrand prod 1/(0.9^2 + (x_i - 0.6)^2) on
    # [-1,1]^d.  The printed relative errors for d = 30, 50, 70, 90 are k
    # times the d = 10 one (k = d/10 blocks) to the printed digits.  A tensor
    # product of k equal blocks with relative error eta has error
    # |(1 + eta)^k - 1|, which is k |eta| to first order; the test checks
    # that first-order growth against the printed values, allowing the
    # second-order term C(k,2) eta^2 and the difference between the printed
    # single-block error and this rule's (1.4304e-4 printed, 1.43058e-4 here).
    printed = {10: 1.4304e-4, 30: 4.2912e-4, 50: 7.1521e-4, 70: 1.0012e-3, 90: 1.2873e-3}
    errs = {}
    for d in printed:
        params = np.concatenate([np.full(d, 1 / 0.45), np.full(d, 0.8)])
        v = B.smolyak_blocked(d, d + 9, "gl_paper", "product_peak", params, 10, "factorised")
        ex = R.exact("product_peak", d, params)
        errs[d] = float(abs((mp.mpf(v) - ex) / ex))
    eta = errs[10]
    assert abs(eta - printed[10]) <= 3e-4 * printed[10]
    for d, p in printed.items():
        k = d // 10
        assert abs(errs[d] - abs((1 - eta) ** k - 1)) <= 1e-9 * errs[d]     # k equal blocks multiply
        slack = comb(k, 2) * eta ** 2 * 1.01 + k * abs(eta - printed[10]) + 0.5e-4 * p
        assert abs(errs[d] - p) <= slack, (d, errs[d], p, slack)


@pytest.mark.parametrize("rule", ["cc", "gl", "tr", "gp"])
def test_oscillatory_rule_is_a_rotation_of_its_phase_cancelled_value(rule):
    """For cos(2 pi w + sum a_i x_i) the rule's value is linear in e^{2 pi i w}:
    with theta = sum a_i / 2 and S its value at w = -theta / 2 pi, the values
    at w = 0 and w = -1/4 are cos(theta) S and sin(theta) S (the rule is
    symmetric about the centre, so its sum of e^{i a (x - 1/2)} is real).  The
    block variant sweeps an oscillatory block once at that w and rotates the
    result; this pins the identity on the oracle's point-by-point sum."""
    import oracle
    rng = np.random.default_rng(23 + len(rule))
    for d, K in ((1, 3), (4, 2), (6, 3)):
        a = rng.uniform(-3.0, 3.0, d)
        th = 0.5 * float(np.sum(a))

        def val(w):
            return oracle.smolyak_points(d, d + K, rule, "oscillatory", np.concatenate([[w], a]))

        r_s, r_re, r_im = val(-th / (2.0 * np.pi)), val(0.0), val(-0.25)
        s = r_s["q"]
        # each sum's rounding (a small multiple of 2^-64 (A + |f(c)|)), the
        # rounding of w = -theta / 2 pi and of cos, sin and the products
        tol = sum(2.0 ** -56 * (r["A"] + abs(r["fc"])) for r in (r_s, r_re, r_im)) + 1e-15 * abs(s) * (1.0 + abs(th))
        assert abs(s) > 1e-3
        assert abs(r_re["q"] - np.cos(th) * s) <= tol, (rule, d, K, r_re["q"], np.cos(th) * s, tol)
        assert abs(r_im["q"] - np.sin(th) * s) <= tol, (rule, d, K, r_im["q"], np.sin(th) * s, tol)
