"""Pins for the oracle's Smolyak values ((2.6)-(2.7), Section 2.1).

The point-by-point sum and the factorised sum are checked against each
other, and both against: a numpy brute force built from independently
constructed rules, polynomial exactness, closed-form integrals where the
rule's truncation error is negligible, values printed in the paper
(Tables 5.6-5.8), and invariants of the definition.
"""
import json
import os
from itertools import product
from math import comb

import mpmath as mp
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle import counts as C
from oracle import reference as R
from paper_2210_14313_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U64 = 2.0 ** -64


# ------------------------------------------------------------- brute force
_GP_CACHE = {}


def _mp_patterson(npts):
    """Gauss-Patterson nodes and weights on [0,1] built without the oracle:
    each extension's new nodes are the roots (mpmath polyroots, 50 digits)
    of the monic polynomial of degree n+1 orthogonal, against the previous
    nodes' polynomial, to every lower degree (monomial basis, exact moments);
    weights from the monomial moment equations at 50 digits."""
    if npts in _GP_CACHE:
        return _GP_CACHE[npts]
    with mp.workdps(50):
        mom = lambda k: mp.mpf(2) / (k + 1) if k % 2 == 0 else mp.mpf(0)

        def pmul(a, b):
            r = [mp.mpf(0)] * (len(a) + len(b) - 1)
            for i, x in enumerate(a):
                for j, y in enumerate(b):
                    r[i + j] += x * y
            return r
        nodes = [mp.mpf(0)]
        while len(nodes) < npts:
            n = len(nodes)
            pi = [mp.mpf(1)]
            for t in nodes:
                pi = pmul(pi, [-t, mp.mpf(1)])
            m = n + 1
            A = mp.matrix(m, m)
            rhs = mp.matrix(m, 1)
            for k in range(m):
                for j in range(m):
                    A[k, j] = sum(c * mom(i + j + k) for i, c in enumerate(pi))
                rhs[k] = -sum(c * mom(i + m + k) for i, c in enumerate(pi))
            # pi is odd and the extension even: keep the non-trivial equations
            idx = [j for j in range(m) if (j - m) % 2 == 0]
            rows = [k for k in range(m) if (k + n + m) % 2 == 0]
            B = mp.matrix(len(rows), len(idx))
            r = mp.matrix(len(rows), 1)
            for a_, k in enumerate(rows):
                for b_, j in enumerate(idx):
                    B[a_, b_] = A[k, j]
                r[a_] = rhs[k]
            cc = mp.lu_solve(B, r)
            coef = [mp.mpf(0)] * m
            for b_, j in enumerate(idx):
                coef[j] = cc[b_]
            roots = mp.polyroots((coef + [mp.mpf(1)])[::-1], maxsteps=400, extraprec=400)
            nodes = sorted(nodes + [mp.re(z) for z in roots])
        V = mp.matrix(npts, npts)
        b = mp.matrix(npts, 1)
        for k in range(npts):
            for i in range(npts):
                V[k, i] = nodes[i] ** k
            b[k] = mom(k)
        w = mp.lu_solve(V, b)
        res = (np.array([float((1 + t) / 2) for t in nodes]), np.array([float(w[i] / 2) for i in range(npts)]))
    _GP_CACHE[npts] = res
    return res


def _numpy_rule(rule, level):
    """1-D rules built without the oracle: numpy's Gauss-Legendre, and
    interpolatory weights from Legendre moments for the Clenshaw-Curtis
    nodes; trapezoid directly; Gauss-Patterson with mpmath."""
    if level == 1:
        return np.array([0.5]), np.array([1.0])
    if rule == "gp":
        return _mp_patterson((1, 3, 3, 7, 7, 7, 15, 15, 15, 15)[level - 1])
    if rule == "gl" or rule == "gl_paper":
        n = 2 * level - 1 if rule == "gl" else level
        t, w = npleg.leggauss(n)
        return (t + 1) / 2, w / 2
    n = 2 ** (level - 1) + 1
    if rule == "tr":
        x = np.linspace(0, 1, n)
        w = np.full(n, 1.0 / (n - 1))
        w[0] = w[-1] = 0.5 / (n - 1)
        return x, w
    x = (1 - np.cos(np.pi * np.arange(n) / (n - 1))) / 2
    V = npleg.legvander(2 * x - 1, n - 1).T      # rows: P_k at the nodes
    rhs = np.zeros(n)
    rhs[0] = 1.0                                 # int_0^1 P_k(2x-1) dx = delta_k0
    return x, np.linalg.solve(V, rhs)


def _f(family, params, X):
    d = X.shape[-1]
    if family == "exp_sum":
        return np.exp(X @ params[:d])
    if family == "oscillatory":
        return np.cos(2 * np.pi * params[0] + X @ params[1:1 + d])
    if family == "corner_peak":
        return (1.0 + X @ params[:d]) ** (-(d + 1))
    if family == "gaussian":
        return np.exp(((X - params[d:2 * d]) ** 2) @ params[:d])
    if family == "oscillatory_quadratic":
        return np.cos(2 * np.pi * params[0] + ((X - params[1 + d:1 + 2 * d]) ** 2) @ params[1:1 + d])
    if family == "oscillatory_quadratic_linear":
        return np.cos(2 * np.pi * params[0] + ((X - params[1 + d:1 + 2 * d]) ** 2) @ params[1:1 + d]
                      + X @ params[1 + 2 * d:1 + 3 * d])
    b, u = params[:d], params[d:2 * d]
    return np.prod(1.0 / (b ** -2 + (X - u) ** 2), axis=-1)


def brute_smolyak(d, q, rule, family, params):
    """(2.6)-(2.7) literally: every window multi-index, every tensor point."""
    total = 0.0
    for l in product(range(1, q + 1), repeat=d):
        s = sum(l)
        if not (q - d + 1 <= s <= q):
            continue
        rules = [_numpy_rule(rule, li) for li in l]
        grids = np.meshgrid(*[r[0] for r in rules], indexing="ij")
        wgts = np.meshgrid(*[r[1] for r in rules], indexing="ij")
        X = np.stack([g.ravel() for g in grids], axis=-1)
        Wt = np.prod(np.stack([g.ravel() for g in wgts], axis=-1), axis=-1)
        coef = (-1) ** (q - s) * comb(d - 1, q - s)
        total += coef * np.sum(Wt * _f(family, params, X))
    return total


SMALL = [(d, q, r, f) for (d, q) in [(1, 3), (2, 3), (2, 5), (3, 5), (3, 6), (4, 6)]
         for r in ("tr", "cc", "gl", "gl_paper", "gp")
         for f in ("exp_sum", "oscillatory", "product_peak", "corner_peak", "gaussian", "oscillatory_quadratic",
                   "oscillatory_quadratic_linear")]


@pytest.mark.parametrize("d,q,rule,family", SMALL)
def test_point_oracle_matches_numpy_brute_force(orc, d, q, rule, family):
    rng = np.random.default_rng(1000 + d * 31 + q)
    params = W.draw_params(rng, family, d, osc_scale=3.0)
    ref = brute_smolyak(d, q, rule, family, params)
    got = orc.smolyak_points(d, q, rule, family, params)
    assert abs(got["q"] - ref) <= 1e-13 * max(1.0, abs(ref)), (got, ref)


# --------------------------------------------------- points vs factorised
def _random_cases(seed, n, d_range, k_range):
    b = W.random_small(seed, n, d_range, k_range, osc_scale=9.0)
    return [(p.d, p.q, p.rule, p.family, b.param_slice(i)) for i, p in enumerate(b.problems)]


@pytest.mark.parametrize("case", _random_cases(7, 40, (1, 12), (0, 5)))
def test_points_match_factorised(orc, case):
    d, q, rule, family, params = case
    pt = orc.smolyak_points(d, q, rule, family, params)
    fq = orc.smolyak_factorised(d, q, rule, family, params)
    tol = 8 * U64 * (pt["A"] + abs(pt["fc"])) + 4e-16 * abs(fq)
    assert abs(pt["q"] - fq) <= tol, (pt, fq, tol)


def _quadratic_cases(seed, n):
    b = W.random_small(seed, n, (1, 8), (0, 6), families=("gaussian", "oscillatory_quadratic",
                                                          "oscillatory_quadratic_linear"), rules=W.ALL_RULES)
    return [(p.d, p.q, p.rule, p.family, b.param_slice(i)) for i, p in enumerate(b.problems)]


@pytest.mark.parametrize("case", _quadratic_cases(8, 24))
def test_points_match_factorised_quadratic_families(orc, case):
    # the factorisation of (2.6) with the quadratic families' factors (the
    # oscillatory quadratic's complex) against the literal point sum
    d, q, rule, family, params = case
    pt = orc.smolyak_points(d, q, rule, family, params)
    fq = orc.smolyak_factorised(d, q, rule, family, params)
    tol = 8 * U64 * (pt["A"] + abs(pt["fc"])) + 4e-16 * max(abs(fq), 1.0)
    assert abs(pt["q"] - fq) <= tol, (pt, fq, tol)


@pytest.mark.parametrize("d,K,rule,family", [(30, 3, "cc", "exp_sum"), (25, 3, "gl", "oscillatory"),
                                             (40, 2, "tr", "product_peak"), (12, 5, "cc", "oscillatory")])
def test_points_match_factorised_medium(orc, d, K, rule, family):
    rng = np.random.default_rng(d * 100 + K)
    params = W.draw_params(rng, family, d)
    pt = orc.smolyak_points(d, d + K, rule, family, params)
    fq = orc.smolyak_factorised(d, d + K, rule, family, params)
    assert abs(pt["q"] - fq) <= 1e-14 * abs(fq) + 8 * U64 * pt["A"]


def test_centred_and_uncentred_agree(orc):
    for fam in ("exp_sum", "oscillatory", "product_peak", "corner_peak"):
        rng = np.random.default_rng(5)
        params = W.draw_params(rng, fam, 6)
        a = orc.smolyak_points(6, 10, "cc", fam, params, centred=True)["q"]
        b = orc.smolyak_points(6, 10, "cc", fam, params, centred=False)["q"]
        assert abs(a - b) < 1e-14 * abs(a)


# ------------------------------------------------------------ corner peak
def test_corner_peak_closed_form_independent():
    # the subset formula against d = 1 by hand and d = 2, 3 by quadrature of
    # the integral with its last coordinate integrated by hand:
    # int_0^1 (s + a x)^-(d+1) dx = (s^-d - (s + a)^-d) / (d a)
    a1 = 0.7
    assert abs(float(R.exact_corner_peak([a1])) - 1.0 / (1.0 + a1)) < 1e-15
    for a in ([0.3, 0.9], [0.2, 0.5, 0.4]):
        d = len(a)
        al = a[-1]

        def f(*x):
            s = 1 + sum(ai * xi for ai, xi in zip(a[:-1], x))
            return (s ** -d - (s + al) ** -d) / (d * al)
        with mp.workdps(20):
            ref = mp.quad(f, *([[0, 1]] * (d - 1)))
        assert abs(float(R.exact_corner_peak(a)) - float(ref)) < 1e-14 * float(ref)


@pytest.mark.parametrize("d,q", [(1, 12), (2, 12), (3, 11)])
def test_corner_peak_converges_to_closed_form(orc, d, q):
    # an analytic integrand: high-level Gauss-Legendre Smolyak sums converge
    rng = np.random.default_rng(77 + d)
    a = W.draw_params(rng, "corner_peak", d)
    got = orc.smolyak_points(d, q, "gl", "corner_peak", a)["q"]
    ex = float(R.exact_corner_peak(a))
    assert abs(got - ex) <= 1e-12 * ex, (got, ex)


def test_rule_integrates_one_exactly(orc):
    # f = 1 (exp-sum with c = 0): the signed combination weights total 1
    for rule in ("tr", "cc", "gl", "gl_paper", "gp"):
        for d, q in [(1, 4), (3, 7), (7, 10), (20, 23)]:
            r = orc.smolyak_points(d, q, rule, "exp_sum", np.zeros(d), centred=False)
            assert abs(r["q"] - 1.0) < 1e-15


# --------------------------------------------------- polynomial exactness
def _level_needed(rule, alpha):
    """Smallest excess e with the level-(e+1) rule exact for degree alpha."""
    deg = {"cc": lambda l: 1 if l == 1 else 2 ** (l - 1) + 1,
           "gl": lambda l: 4 * l - 3,
           "gl_paper": lambda l: 2 * l - 1,
           "gp": lambda l: (1, 5, 5, 11, 11, 11, 23, 23, 23, 23)[l - 1] if l <= 10 else 23,
           "tr": lambda l: 1}[rule]
    e = 0
    while deg(e + 1) < alpha:
        e += 1
        if e > 30:
            return None
    return e


@pytest.mark.parametrize("rule", ["cc", "gl", "gl_paper", "gp"])
def test_polynomial_exactness(orc, rule):
    # Smolyak's rule integrates prod (x_i - s)^alpha_i exactly when the levels
    # that integrate each factor exactly fit into the excess budget K.
    rng = np.random.default_rng(3)
    d, K = 4, 4
    tried_in = tried_out = 0
    # random degree vectors, plus every even vector just outside the budget
    cands = [rng.integers(0, 9, d) for _ in range(200)]
    cands += [np.array(a) for a in product(range(0, 11, 2), repeat=d)
              if sum(_level_needed(rule, x) for x in a) == K + 1][:12]
    for alpha in cands:
        need = sum(_level_needed(rule, a) for a in alpha)
        s = 0.5 if (need == K + 1 or rng.random() < 0.5) else 0.0
        exact = 1.0
        for a in alpha:
            exact *= ((1 - s) ** (a + 1) - (0 - s) ** (a + 1)) / (a + 1)
        got = orc.smolyak_points(d, d + K, rule, "monomial", np.concatenate([alpha, [s]]))["q"]
        if need <= K:
            assert abs(got - exact) <= 1e-15 * max(1, abs(exact)), (alpha, s)
            tried_in += 1
        elif s == 0.5 and all(a % 2 == 0 for a in alpha) and need == K + 1:
            # just outside the exactness set: must NOT be exact
            assert abs(got - exact) > 1e-13 * abs(exact), (alpha, got, exact)
            tried_out += 1
    assert tried_in > 10 and tried_out >= 1


# -------------------------------------------------------- closed forms
def test_closed_form_where_truncation_is_negligible(orc):
    # d=100, q=105, Clenshaw-Curtis, oscillatory: truncation far below 1e-12
    b = W.precision_d100()
    p = b.problems[0]
    v = orc.smolyak_factorised(p.d, p.q, p.rule, p.family, b.param_slice(0))
    ex = float(R.exact(p.family, p.d, b.param_slice(0)))
    assert abs(v - ex) < 1e-13 * abs(ex)
    # d=1000, q=1003, Gauss-Legendre, exp(sum c_i x_i / d)
    b = W.high_dim_d1000(rules=("gl",))
    p = b.problems[0]
    v = orc.smolyak_factorised(p.d, p.q, p.rule, p.family, b.param_slice(0))
    ex = float(R.exact(p.family, p.d, b.param_slice(0)))
    assert abs(v - ex) < 1e-14 * abs(ex)
    # d=10, q=14, Clenshaw-Curtis exp-sum: truncation is visible but small
    b = W.plain_exp_d10()
    p = b.problems[0]
    v = orc.smolyak_points(p.d, p.q, p.rule, p.family, b.param_slice(0))["q"]
    ex = float(R.exact(p.family, p.d, b.param_slice(0)))
    assert 1e-12 < abs(v - ex) / ex < 1e-7


# ------------------------------------------------------- paper's values
def _paper_params(integrand, d):
    if integrand == "exp_alt":
        return "exp_sum", np.array([2.0 * (-1) ** i for i in range(d)])
    if integrand == "cos_sum":
        return "oscillatory", np.concatenate([[1 - d / (2 * np.pi)], np.full(d, 2.0)])
    return "product_peak", np.concatenate([np.full(d, 1 / 0.45), np.full(d, 0.8)])


def _same_to_5_digits(a, b):
    ea = int(np.floor(np.log10(abs(b))))
    return abs(a - b) <= 1.01 * 10.0 ** (ea - 4)


def test_paper_tables_5_6_to_5_8(orc):
    g = json.load(open(os.path.join(GOLDEN, "paper_tables_5_6_to_5_8.json")))
    for row in g["rows"]:
        d, N = row["d"], row["N"]
        fam, params = _paper_params(row["integrand"], d)
        q = d + N - 1
        ex = R.exact(fam, d, params)
        v = orc.smolyak_factorised(d, q, "gl_paper", fam, params)
        rel = float(abs((mp.mpf(v) - ex) / ex))
        assert _same_to_5_digits(rel, row["rel_err"]), (row, rel)
        if d == 5:
            vp = orc.smolyak_points(d, q, "gl_paper", fam, params)["q"]
            relp = float(abs((mp.mpf(vp) - ex) / ex))
            assert _same_to_5_digits(relp, row["rel_err"]), (row, relp)


# ----------------------------------------------------------- invariants
def test_permutation_invariance(orc):
    rng = np.random.default_rng(11)
    d = 7
    for fam in ("exp_sum", "oscillatory", "product_peak"):
        params = W.draw_params(rng, fam, d)
        perm = rng.permutation(d)
        if fam == "exp_sum":
            pp = params[perm]
        elif fam == "oscillatory":
            pp = np.concatenate([[params[0]], params[1:][perm]])
        else:
            pp = np.concatenate([params[:d][perm], params[d:][perm]])
        a = orc.smolyak_points(d, d + 4, "cc", fam, params)["q"]
        b = orc.smolyak_points(d, d + 4, "cc", fam, pp)["q"]
        assert abs(a - b) < 1e-15 * abs(a)


def test_dimension_padding(orc):
    # a coordinate whose factor is constant changes nothing once q grows by 1
    rng = np.random.default_rng(12)
    d, K = 6, 4
    c = W.draw_params(rng, "exp_sum", d)
    a = orc.smolyak_points(d, d + K, "gl", "exp_sum", c)["q"]
    b = orc.smolyak_points(d + 1, d + 1 + K, "gl", "exp_sum", np.concatenate([c, [0.0]]))["q"]
    assert abs(a - b) < 1e-15 * abs(a)
    osc = W.draw_params(rng, "oscillatory", d)
    a = orc.smolyak_points(d, d + K, "cc", "oscillatory", osc)["q"]
    b = orc.smolyak_points(d + 1, d + 1 + K, "cc", "oscillatory", np.concatenate([osc, [0.0]]))["q"]
    assert abs(a - b) < 1e-14 * max(abs(a), 1e-3)


def test_one_dimension_is_the_1d_rule(orc):
    for rule in ("tr", "cc", "gl", "gl_paper", "gp"):
        for q in (1, 3, 6):
            c = np.array([0.7])
            x, w = orc.rule(rule, q)
            ref = float(np.sum(w * np.exp(0.7 * x)))
            got = orc.smolyak_points(1, q, rule, "exp_sum", c)["q"]
            assert abs(got - ref) < 1e-15 * ref


def test_two_dimensions_is_the_two_term_formula(orc):
    # d = 2: (2.6) has only |l| = q (coefficient +1) and |l| = q-1 (coefficient -1)
    rng = np.random.default_rng(4)
    c = W.draw_params(rng, "exp_sum", 2)
    q = 6
    ref = 0.0
    for s, sign in ((q, 1.0), (q - 1, -1.0)):
        for l1 in range(1, s):
            x1, w1 = orc.rule("cc", l1)
            x2, w2 = orc.rule("cc", s - l1)
            ref += sign * np.sum(np.outer(w1 * np.exp(c[0] * x1), w2 * np.exp(c[1] * x2)))
    got = orc.smolyak_points(2, q, "cc", "exp_sum", c)["q"]
    assert abs(got - ref) < 1e-15 * abs(ref)


# -------------------------------------------------------------- gradients
def test_factorised_gradient_matches_finite_differences(orc):
    rng = np.random.default_rng(21)
    for fam, rule, d, K in [("oscillatory", "cc", 8, 3), ("exp_sum", "gl", 6, 4), ("product_peak", "cc", 5, 3),
                            ("gaussian", "gp", 5, 4), ("oscillatory_quadratic", "gl", 4, 3),
                            ("oscillatory_quadratic_linear", "cc", 4, 3)]:
        params = W.draw_params(rng, fam, d)
        g = orc.smolyak_factorised_grad(d, d + K, rule, fam, params)
        h = 1e-6
        for k in range(len(params)):
            pp, pm = params.copy(), params.copy()
            pp[k] += h
            pm[k] -= h
            hp = orc.smolyak_factorised_hilo(d, d + K, rule, fam, pp)
            hm = orc.smolyak_factorised_hilo(d, d + K, rule, fam, pm)
            fd = ((hp[0] - hm[0]) + (hp[1] - hm[1])) / (2 * h)
            assert abs(fd - g[k]) <= 1e-8 * max(1.0, abs(g[k])), (fam, k, fd, g[k])


def test_factorised_gradient_matches_closed_form(orc):
    b = W.gradient_osc_d200(n=2)
    for i, p in enumerate(b.problems):
        params = b.param_slice(i)
        g = orc.smolyak_factorised_grad(p.d, p.q, p.rule, p.family, params)
        ge = R.exact_grad_oscillatory(params[0], params[1:])
        np.testing.assert_allclose(g, ge, rtol=1e-12, atol=1e-14 * np.max(np.abs(ge)))


# ------------------------------------------------ quadratic exponentials
@pytest.mark.parametrize("family", ["gaussian", "oscillatory_quadratic", "oscillatory_quadratic_linear"])
def test_quadratic_families_converge_to_closed_form(orc, family):
    # entire integrands: high-level Gauss-Legendre sums reach the erf closed
    # forms (checked against mpmath quadrature in one dimension)
    rng = np.random.default_rng(31)
    for d, q in [(1, 9), (2, 11), (3, 11)]:
        prm = W.draw_params(rng, family, d)
        got = orc.smolyak_points(d, q, "gl", family, prm)["q"]
        ex = float(R.exact(family, d, prm))
        assert abs(got - ex) <= 1e-12 * max(abs(ex), 0 if family == "gaussian" else 1e-3), (d, got, ex)
    c, u, a, w = 1.7, 0.3, -2.2, 0.4
    with mp.workdps(30):
        q1 = mp.quad(lambda x: mp.exp(c * (x - u) ** 2), [0, 1])
        q2 = mp.quad(lambda x: mp.cos(2 * mp.pi * w + a * (x - u) ** 2), [0, 1])
    assert abs(float(R.exact_gaussian([c], [u])) - float(q1)) < 1e-15 * float(q1)
    assert abs(float(R.exact_oscillatory_quadratic(w, [a], [u])) - float(q2)) < 1e-15


def test_paper_table_4_1_first_row(orc):
    g = json.load(open(os.path.join(GOLDEN, "paper_table_4_1.json")))
    for row in g["rows"]:
        d, q = row["d"], row["q"]
        prm = np.array(row["params"], dtype=np.float64)
        v = orc.smolyak_points(d, d + q - 1, g["rule"], g["family"], prm)["q"]
        vf = orc.smolyak_factorised(d, d + q - 1, g["rule"], g["family"], prm)
        ex = R.exact(g["family"], d, prm)
        for val in (v, vf):
            rel = float(abs((mp.mpf(val) - ex) / ex))
            assert _same_to_5_digits(rel, row["rel_err"]), (row, rel)


# ------------------------------------- quadratic phase with a linear term
def test_linear_term_closed_form_against_quadrature():
    # the completed-square closed form of int_0^1 e^{i (a (x-u)^2 + c x)} dx
    # against mpmath's quadrature, including a = 0 (the linear oscillatory
    # factor) and a small a with a far-off completed centre
    for a, u, c in [(-2.2, 0.3, 1.1), (3.0, 0.9, -4.0), (0.0, 0.5, 2.5), (1e-3, 0.2, 0.7), (40.0, 0.5, 0.0)]:
        with mp.workdps(30):
            qre = mp.quad(lambda x: mp.cos(a * (x - u) ** 2 + c * x), [0, 1])
            qim = mp.quad(lambda x: mp.sin(a * (x - u) ** 2 + c * x), [0, 1])
        z = R._quad_linear_1d(a, u, c)
        assert abs(complex(z) - complex(qre, qim)) < 1e-15, (a, u, c)


@pytest.mark.parametrize("rule", ["cc", "gl", "gp"])
def test_linear_term_reduces_to_the_other_oscillatory_families(orc, rule):
    # c = 0 is the oscillatory quadratic; a = 0 is the linear oscillatory
    # family (its own real-surplus code path in the oracle) with c as its
    # coefficients, u unused
    rng = np.random.default_rng(61)
    for d, K in [(1, 4), (3, 3), (6, 2), (20, 4)]:
        p = W.draw_params(rng, "oscillatory_quadratic_linear", d)
        w, a, u, c = p[0], p[1:1 + d], p[1 + d:1 + 2 * d], p[1 + 2 * d:]
        q0 = np.concatenate([[w], a, u, np.zeros(d)])
        v0 = orc.smolyak_factorised(d, d + K, rule, "oscillatory_quadratic_linear", q0)
        assert v0 == orc.smolyak_factorised(d, d + K, rule, "oscillatory_quadratic", p[:1 + 2 * d])
        q1 = np.concatenate([[w], np.zeros(d), u, c])
        v1 = orc.smolyak_factorised(d, d + K, rule, "oscillatory_quadratic_linear", q1)
        v2 = orc.smolyak_factorised(d, d + K, rule, "oscillatory", np.concatenate([[w], c]))
        assert abs(v1 - v2) <= 1e-15 * max(1.0, abs(v2)), (d, K, v1, v2)
        if d <= 6:
            pt = orc.smolyak_points(d, d + K, rule, "oscillatory_quadratic_linear", q1)["q"]
            po = orc.smolyak_points(d, d + K, rule, "oscillatory", np.concatenate([[w], c]))["q"]
            assert abs(pt - po) <= 1e-15 * max(1.0, abs(po))
