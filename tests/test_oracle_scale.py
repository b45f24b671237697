"""Pins for the oracle's accuracy scale (oracle.accuracy_scale).

For the oscillatory families the scale of a result is the modulus |S| of the
complex Smolyak sum (2.6) of e^{i phase(x)}, formed by the oracle as
sqrt(Q(w)^2 + Q(w - 1/4)^2).  It is pinned here by things that do not use
that formula: independence of w, the one-dimensional rule written out with
numpy's Gauss-Legendre nodes, and the modulus of the exact integral
(a product of |sinc| factors) where the rule's truncation error is
negligible.  For the other families the scale is |Q|.
"""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from paper_2210_14313_amd import workloads as W


def test_scale_of_non_oscillatory_is_abs(orc):
    b = W.random_small(31, 24, d_range=(1, 8), k_range=(0, 4), families=("exp_sum", "product_peak"))
    ref = orc.batch_factorised(b)
    assert np.array_equal(orc.accuracy_scale(b, ref), np.abs(ref))


@pytest.mark.parametrize("family", ["oscillatory", "oscillatory_quadratic", "oscillatory_quadratic_linear"])
def test_modulus_does_not_depend_on_w(orc, family):
    b = W.random_small(32, 16, d_range=(1, 30), k_range=(0, 5), families=(family,))
    ref = orc.batch_factorised(b)
    s1 = orc.accuracy_scale(b, ref)
    for i, p in enumerate(b.problems):
        b.params[p.param_offset] += 0.3719
    ref2 = orc.batch_factorised(b)
    s2 = orc.accuracy_scale(b, ref2)
    assert np.max(np.abs(s1 - s2) / s1) <= 1e-14
    # Q itself does change with w, and never exceeds the modulus
    assert np.max(np.abs(ref - ref2)) > 1e-3
    assert np.all(np.abs(ref) <= s1 * (1 + 1e-15)) and np.all(np.abs(ref2) <= s2 * (1 + 1e-15))


@pytest.mark.parametrize("q", [1, 2, 5, 9])
def test_one_dimension_gauss_legendre_paper_mode(orc, q):
    # d = 1: (2.6) is the level-q rule itself; paper-mode Gauss-Legendre has
    # q nodes, taken here from numpy and mapped to [0,1]
    w0, a = 0.137, 7.3
    x, wt = npleg.leggauss(q)
    x, wt = (x + 1) / 2, wt / 2
    S = np.sum(wt * np.exp(1j * a * x))
    ref = orc.smolyak_factorised(1, q, "gl_paper", "oscillatory", np.array([w0, a]))
    assert abs(ref - np.real(np.exp(2j * np.pi * w0) * S)) <= 1e-14
    got = orc.accuracy_scale_one(1, q, "gl_paper", "oscillatory", np.array([w0, a]), ref)
    assert abs(got - abs(S)) <= 1e-14 * abs(S)


def test_modulus_of_exact_integral_at_d100(orc):
    # d = 100, q = 105, Clenshaw-Curtis, a_i ~ U(0,1) 9/d: the rule's
    # truncation error is ~1e-15, so |S| is the modulus of the exact integral
    # prod_t |(e^{i a_t} - 1)/(i a_t)| = prod_t |sinc(a_t/2)|
    b = W.precision_d100()
    i = [k for k, p in enumerate(b.problems) if p.family == "oscillatory"][0]
    p = b.problems[i]
    prm = b.param_slice(i)
    a = prm[1:]
    exact_mod = float(np.prod(np.abs(np.sin(a / 2) / (a / 2))))
    ref = orc.smolyak_factorised(p.d, p.q, p.rule, p.family, prm)
    got = orc.accuracy_scale_one(p.d, p.q, p.rule, p.family, prm, ref)
    assert abs(got - exact_mod) <= 1e-13 * exact_mod
    one = b.subset([i])
    assert abs(orc.accuracy_scale(one, np.array([ref]))[0] - got) <= 1e-15 * got
