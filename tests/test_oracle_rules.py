"""Pins for the oracle's 1-D rules (Section 2.2, (2.10)-(2.13)), on [0,1].

Each check is tied to something other than the oracle's own formula: a
textbook value, numpy's Gauss-Legendre routine, exact moments of monomials,
or a structural property (nesting, symmetry).
"""
import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss

RULES = ["tr", "cc", "gl", "gl_paper", "gp"]


@pytest.mark.parametrize("rule", RULES)
@pytest.mark.parametrize("level", range(1, 9))
def test_weights_sum_to_one_and_symmetry(orc, rule, level):
    x, w = orc.rule(rule, level)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.all(np.diff(x) > 0)
    assert np.max(np.abs(x + x[::-1] - 1.0)) < 1e-15
    assert np.max(np.abs(w - w[::-1])) < 1e-15
    if rule != "tr":
        assert np.all(w > 0)


def test_level_one_is_midpoint(orc):
    for r in RULES:
        x, w = orc.rule(r, 1)
        assert list(x) == [0.5] and list(w) == [1.0]


def test_textbook_small_rules(orc):
    # Clenshaw-Curtis with 3 points = Simpson's rule
    x, w = orc.rule("cc", 2)
    np.testing.assert_allclose(x, [0, 0.5, 1], atol=1e-16)
    np.testing.assert_allclose(w, [1 / 6, 2 / 3, 1 / 6], rtol=1e-15)
    # trapezoidal with 3 points
    x, w = orc.rule("tr", 2)
    np.testing.assert_allclose(w, [0.25, 0.5, 0.25], rtol=0)
    # 3-point Gauss-Legendre on [0,1]: nodes 1/2 -+ sqrt(3/5)/2, weights 5/18, 4/9, 5/18
    x, w = orc.rule("gl", 2)
    np.testing.assert_allclose(x, [0.5 - np.sqrt(0.6) / 2, 0.5, 0.5 + np.sqrt(0.6) / 2], rtol=1e-15)
    np.testing.assert_allclose(w, [5 / 18, 4 / 9, 5 / 18], rtol=1e-15)


@pytest.mark.parametrize("n", range(1, 21))
def test_gauss_legendre_matches_numpy(orc, n):
    # level l of the paper's count has n_l = l points
    x, w = orc.rule("gl_paper", n)
    t, om = leggauss(n)
    np.testing.assert_allclose(x, (t + 1) / 2, rtol=0, atol=2e-15)
    # numpy computes its weights in double precision (about 1e-13 relative)
    np.testing.assert_allclose(w, om / 2, rtol=1e-13)
    if n % 2 == 1:
        lvl = (n + 1) // 2
        x2, w2 = orc.rule("gl", lvl)
        np.testing.assert_allclose(x2, x, atol=0)


def _moment_err(x, w, k):
    return abs(np.sum(w * x ** k) - 1.0 / (k + 1))


@pytest.mark.parametrize("level", range(2, 9))
def test_clenshaw_curtis_exactness_degree(orc, level):
    # an n-point symmetric interpolatory rule (n odd) is exact up to degree n
    x, w = orc.rule("cc", level)
    n = len(x)
    for k in range(0, n + 1):
        assert _moment_err(x, w, k) < 1e-14, (level, k)
    if level <= 5:     # beyond that the degree-(n+1) error is below double rounding
        assert _moment_err(x, w, n + 1) > 1e-15


@pytest.mark.parametrize("level", range(2, 8))
def test_gauss_legendre_exactness_degree(orc, level):
    x, w = orc.rule("gl", level)
    n = len(x)
    for k in range(0, 2 * n):
        assert _moment_err(x, w, k) < 1e-14
    if level <= 5:     # beyond that the degree-2n error is below double rounding
        assert _moment_err(x, w, 2 * n) > 1e-15


@pytest.mark.parametrize("level", range(2, 8))
def test_trapezoid_error_on_square(orc, level):
    # composite trapezoid with spacing h integrates x^2 on [0,1] with error h^2/6
    x, w = orc.rule("tr", level)
    h = 1.0 / (len(x) - 1)
    assert abs(np.sum(w * x) - 0.5) < 1e-15
    assert abs((np.sum(w * x ** 2) - 1 / 3) - h * h / 6) < 1e-15


@pytest.mark.parametrize("rule", ["tr", "cc", "gp"])
def test_nested_rules_are_nested(orc, rule):
    for level in range(1, 8):
        a, _ = orc.rule(rule, level)
        b, _ = orc.rule(rule, level + 1)
        for v in a:
            assert np.min(np.abs(b - v)) < 1e-15


@pytest.mark.parametrize("rule", ["gl", "gl_paper"])
def test_gauss_legendre_levels_share_only_the_centre(orc, rule):
    xs = [orc.rule(rule, l)[0] for l in range(1, 13)]
    for i in range(len(xs)):
        for j in range(i + 1, len(xs)):
            diff = np.abs(xs[i][:, None] - xs[j][None, :])
            close = diff < 1e-9
            for a, b in zip(*np.nonzero(close)):
                assert abs(xs[i][a] - 0.5) < 1e-15 and abs(xs[j][b] - 0.5) < 1e-15


# ------------------------------------------------------ Gauss-Patterson
def test_gauss_patterson_level_map_of_section_5_4(orc):
    # Section 5.4 lists, for the Gauss-Patterson rule, q = 1..10 <-> N =
    # 1, 3, 3, 7, 7, 7, 15, 15, 15, 15
    assert [orc.rule_npoints("gp", l) for l in range(1, 11)] == [1, 3, 3, 7, 7, 7, 15, 15, 15, 15]
    assert orc.rule_npoints("gp", 11) == -1


def test_gauss_patterson_three_points_is_gauss(orc):
    # the first Patterson extension of the midpoint is the 3-point Gauss rule
    x, w = orc.rule("gp", 2)
    t = np.sqrt(0.6)
    assert np.max(np.abs(x - np.array([(1 - t) / 2, 0.5, (1 + t) / 2]))) < 1e-16
    assert np.max(np.abs(w - np.array([5, 8, 5]) / 18.0)) < 1e-16


@pytest.mark.parametrize("level,degree", [(2, 5), (4, 11), (7, 23)])
def test_gauss_patterson_exactness_degree(orc, level, degree):
    # Kronrod-Patterson extensions: 3 points exact to degree 5, 7 points to
    # 3*3 + 2 = 11, 15 points to 3*7 + 2 = 23; with the nesting below this
    # fixes each rule uniquely (the extension of a rule by n + 1 nodes
    # reaching that degree is unique)
    x, w = orc.rule("gp", level)
    for k in range(degree + 1):
        assert _moment_err(x, w, k) < 5e-16, (level, k)
    # one degree more (even, centred) is not exact
    c = np.sum(w * (x - 0.5) ** (degree + 1))
    exact = 2 * 0.5 ** (degree + 2) / (degree + 2)
    assert abs(c - exact) > 1e-10 * exact
