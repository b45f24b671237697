"""The host-side box map (api.box_to_unit): an integrand on [lo, hi]^d
rewritten on the unit cube of the rule, integral = factor x unit-cube
integral.  Checked per family against the box integral computed
independently: closed forms on the box (exp-sum, oscillatory,
product-peak), products of one-dimensional quadratures (the quadratic
families), and a two-dimensional quadrature (corner-peak), each against the
oracle's closed form of the mapped unit-cube integrand (CPU)."""
import mpmath as mp
import numpy as np
import pytest

from oracle import reference as R
from paper_2210_14313_amd import api, workloads as W


def _boxes(d, rng):
    yield -1.0, 1.0
    lo = rng.uniform(-1.5, 0.5, d)
    yield lo, lo + rng.uniform(0.3, 2.0, d)


def _box_exact(family, p, d, lo, hi):
    lo = np.broadcast_to(np.asarray(lo, dtype=float), (d,))
    hi = np.broadcast_to(np.asarray(hi, dtype=float), (d,))
    if family == "exp_sum":
        r = mp.mpf(1)
        for c, a, b in zip(p[:d], lo, hi):
            c, a, b = mp.mpf(c), mp.mpf(a), mp.mpf(b)
            r *= (mp.exp(c * b) - mp.exp(c * a)) / c
        return r
    if family == "oscillatory":
        z = mp.expj(2 * mp.pi * mp.mpf(p[0]))
        for c, a, b in zip(p[1:1 + d], lo, hi):
            c, a, b = mp.mpf(c), mp.mpf(a), mp.mpf(b)
            z *= (mp.expj(c * b) - mp.expj(c * a)) / (1j * c)
        return mp.re(z)
    if family == "product_peak":
        r = mp.mpf(1)
        for bb, u, a, b in zip(p[:d], p[d:2 * d], lo, hi):
            bb, u, a, b = mp.mpf(bb), mp.mpf(u), mp.mpf(a), mp.mpf(b)
            r *= bb * (mp.atan(bb * (b - u)) - mp.atan(bb * (a - u)))
        return r
    if family == "gaussian":
        r = mp.mpf(1)
        for c, u, a, b in zip(p[:d], p[d:2 * d], lo, hi):
            r *= mp.quad(lambda x: mp.exp(c * (x - u) ** 2), [a, b])
        return r
    if family in ("oscillatory_quadratic", "oscillatory_quadratic_linear"):
        lin = p[1 + 2 * d:1 + 3 * d] if family == "oscillatory_quadratic_linear" else np.zeros(d)
        z = mp.expj(2 * mp.pi * mp.mpf(p[0]))
        for c, u, l, a, b in zip(p[1:1 + d], p[1 + d:1 + 2 * d], lin, lo, hi):
            re = mp.quad(lambda x: mp.cos(c * (x - u) ** 2 + l * x), [a, b])
            im = mp.quad(lambda x: mp.sin(c * (x - u) ** 2 + l * x), [a, b])
            z *= mp.mpc(re, im)
        return mp.re(z)
    if family == "corner_peak":
        assert d == 2
        return mp.quad(lambda x, y: (1 + p[0] * x + p[1] * y) ** -3, [lo[0], hi[0]], [lo[1], hi[1]])
    raise ValueError(family)


@pytest.mark.parametrize("family", ["exp_sum", "oscillatory", "product_peak", "gaussian", "oscillatory_quadratic",
                                    "oscillatory_quadratic_linear", "corner_peak"])
def test_box_map_matches_the_box_integral(family):
    rng = np.random.default_rng(len(family))
    d = 2 if family == "corner_peak" else 3
    for trial in range(3):
        p = W.draw_params(rng, family, d)
        for lo, hi in _boxes(d, rng):
            if family == "corner_peak":
                lo, hi = np.abs(lo), np.abs(lo) + 0.7      # keep 1 + a.x away from zero
            up, factor, frel = api.box_to_unit(family, p, d, lo, hi)
            assert up.shape == p.shape
            got = mp.mpf(factor) * R.exact(family, d, up)
            ref = _box_exact(family, p, d, lo, hi)
            scale = abs(ref) if family not in ("oscillatory", "oscillatory_quadratic",
                                               "oscillatory_quadratic_linear") else max(abs(ref), 1e-2)
            assert abs(got - ref) <= 1e-13 * scale, (family, trial, float(got), float(ref))
            assert 0 <= frel < 1e-13


def test_box_map_paper_domains():
    # (4.1)'s exp(5 x1^2 + 5 x2^2) on [-1,1]^2 is the gaussian c = 20, u = 1/2
    # on the unit cube times the area 4; (4.2)'s sine on [-1,1]^3 is the
    # oscillatory quadratic with a linear term, w = 3/4 - 5/(2 pi),
    # a = (40, 20, 0), u = 1/2, c = (0, 0, 10), times the volume 8
    up, f, _ = api.box_to_unit("gaussian", [5.0, 5.0, 0.0, 0.0], 2, -1.0, 1.0)
    assert list(up) == [20.0, 20.0, 0.5, 0.5] and f == 4.0
    p = np.array([0.75, 10.0, 5.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 5.0])
    up, f, _ = api.box_to_unit("oscillatory_quadratic_linear", p, 3, -1.0, 1.0)
    assert f == 8.0
    np.testing.assert_allclose(up, [0.75 - 5.0 / (2 * np.pi), 40, 20, 0, 0.5, 0.5, 0.5, 0, 0, 10], rtol=0,
                               atol=1e-15)


def test_box_map_rejects_empty_boxes():
    with pytest.raises(ValueError):
        api.box_to_unit("exp_sum", [1.0, 2.0], 2, [0.0, 1.0], [1.0, 1.0])
    with pytest.raises(ValueError):
        api.box_to_unit("corner_peak", [1.0, 1.0], 2, -2.0, 1.0)
