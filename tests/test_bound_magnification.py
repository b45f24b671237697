"""The magnification factor of the a-priori rounding bound (CPU).

The read-out bounds the coefficient sum up to degree K of every partial
product of the coordinates' surplus polynomials delta_t(z) = 1 + sum_e
delta_t[e] z^e by T_K(m) = sum_{j <= K} m^j / j!, m = sum_t sum_e
|delta_t[e]|, evaluated on the device by Horner in FP32 and raised by
1 + 4 (K + 1) 2^-24 (m first rounded up on its conversion to FP32).  These
tests check the claim on random real and complex polynomials (every subset
product, brute force over small sets), that T_K never exceeds exp(m), and the
FP32 evaluation with its margin against the exact value.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest


def _trunc_mul(a, b, K):
    r = np.zeros(K + 1, dtype=a.dtype)
    for i in range(K + 1):
        r[i:] += a[i] * b[:K + 1 - i]
    return r


def _t_k(m, K):
    return sum(m ** j / math.factorial(j) for j in range(K + 1))


@pytest.mark.parametrize("K", [0, 1, 2, 4, 6, 8])
@pytest.mark.parametrize("complex_", [False, True])
def test_every_subset_product_within_truncated_exponential(K, complex_):
    rng = np.random.default_rng(100 + K + 50 * complex_)
    for trial in range(20):
        n = int(rng.integers(1, 7))
        scale = 10.0 ** rng.uniform(-2, 0.7)
        polys = []
        for _ in range(n):
            p = np.zeros(K + 1, dtype=complex if complex_ else float)
            p[0] = 1.0
            c = rng.normal(size=K) * scale
            if complex_:
                c = c + 1j * rng.normal(size=K) * scale
            p[1:] = c
            polys.append(p)
        # the device sums |Re| + |Im| for complex surpluses (at least the modulus)
        m = sum(float(np.sum(np.abs(p[1:].real) + np.abs(p[1:].imag))) for p in polys)
        tk = _t_k(m, K)
        assert tk <= math.exp(m) * (1 + 1e-12)
        for r in range(n + 1):
            for sub in itertools.combinations(range(n), r):
                acc = np.zeros(K + 1, dtype=polys[0].dtype)
                acc[0] = 1.0
                for t in sub:
                    acc = _trunc_mul(acc, polys[t], K)
                assert float(np.sum(np.abs(acc))) <= tk * (1 + 1e-12), (K, trial, sub)


def test_bound_is_attained_by_one_coordinate():
    # one polynomial 1 + m z: coefficient sum 1 + m = T_1(m)
    for m in (0.0, 0.3, 2.0, 17.0):
        p = np.array([1.0, m])
        assert float(np.sum(np.abs(p))) == pytest.approx(_t_k(m, 1))


def _fma32(a, b, c):
    # float32 inputs: the product is exact in float64, the sum rounded there
    # and then to float32 (within one unit of a fused operation)
    return np.float32(float(a) * float(b) + float(c))


@pytest.mark.parametrize("K", [0, 1, 2, 3, 4, 5, 6, 7, 8])
def test_fp32_horner_with_margin_is_an_upper_bound(K):
    rng = np.random.default_rng(7 + K)
    ms = np.concatenate([[0.0, 1e-30, 1e-8, 0.5, 1.0, 3.7, 17.56, 100.0, 1e4],
                         10.0 ** rng.uniform(-6, 4, 200)])
    for m in ms:
        mf = np.float32(np.float32(m) * np.float32(1.0 + 2.0 ** -22))
        r = np.float32(1.0)
        for j in range(K, 0, -1):
            r = _fma32(np.float32(mf * np.float32(np.float32(1.0) / np.float32(j))), r, np.float32(1.0))
        bound = float(r) * (1.0 + 4 * (K + 1) * 2.0 ** -24)
        exact = sum(Fraction(m) ** j / math.factorial(j) for j in range(K + 1))
        assert Fraction(bound) >= exact, (K, m, bound, float(exact))
        # and not loose: within 1e-5 relative of the exact value
        assert bound <= float(exact) * (1 + 1e-5), (K, m)
