"""Block (tensor-product) variant of the sparse-grid rule -- TEST
INFRASTRUCTURE ONLY (tests, smoke and the benchmark's CPU leg).

Algorithm 3.3 reduces the dimension m coordinates at a time (stage 1) and
then s at a time (stage 2), via the Fubini splitting (3.8)-(3.11).  Carried
out exactly with the shared budget of (3.9), that only regroups the sum of
(2.6); the errors the paper reports for m > 1 (Tables 4.7-4.9, 5.1-5.4)
grow in proportion to d/m instead, which is the behaviour of a tensor
product of m-dimensional sparse grids.  This module computes that rule:

* the coordinates are cut into consecutive blocks of m (the last block
  shorter when m does not divide d; stage 2's step s then only regroups
  the last block's sum and does not change the value);
* block b, of dimension d_b, gets its own sparse grid of level
  q_b = d_b + (q - d) in (2.6), i.e. the same excess budget K = q - d;
* the rule is the tensor product of the block rules.

For the product-form families the integrand factors over the blocks, so
the value is the product of the blocks' values: exp-sum, product-peak,
gaussian and monomial directly; oscillatory through
cos(2 pi w + sum_t a_t x_t) = Re(e^{2 pi i w} prod_b e^{i sum_{t in b} a_t x_t}),
where the block value C_b = A_b(cos theta_b) + i A_b(sin theta_b) and
A_b(sin theta_b) = A_b(cos(theta_b - pi/2)) is the oscillatory block with
w = -1/4; the oscillatory quadratic the same way, with
theta_b = sum_{t in b} a_t (x_t - u_t)^2 (plus sum_{t in b} c_t x_t with
the linear term).  Each block value comes from the oracle's plain Smolyak sum
(point by point, or factorised in binary128), and the product is formed in
mpmath at 40 digits.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np


def blocks(d: int, m: int):
    """(start, length) of the consecutive coordinate blocks of size m."""
    if d < 1 or m < 1:
        raise ValueError("d and m must be >= 1")
    return [(s, min(m, d - s)) for s in range(0, d, m)]


def block_params(family: str, params, d: int, start: int, length: int, w_override=None) -> np.ndarray:
    """Parameters of the block integrand (coordinates start..start+length-1)
    in the family's layout."""
    p = np.asarray(params, dtype=np.float64)
    sl = slice(start, start + length)
    if family in ("exp_sum", "corner_peak"):
        return p[sl].copy()
    if family == "oscillatory":
        w = p[0] if w_override is None else w_override
        return np.concatenate([[w], p[1:][sl]])
    if family in ("product_peak", "gaussian"):
        return np.concatenate([p[:d][sl], p[d:2 * d][sl]])
    if family == "monomial":
        return np.concatenate([p[:d][sl], [p[d]]])
    if family == "oscillatory_quadratic":
        w = p[0] if w_override is None else w_override
        return np.concatenate([[w], p[1:1 + d][sl], p[1 + d:1 + 2 * d][sl]])
    if family == "oscillatory_quadratic_linear":
        w = p[0] if w_override is None else w_override
        return np.concatenate([[w], p[1:1 + d][sl], p[1 + d:1 + 2 * d][sl], p[1 + 2 * d:1 + 3 * d][sl]])
    raise ValueError(family)


def smolyak_blocked(d: int, q: int, rule: str, family: str, params, m: int, method: str = "factorised") -> float:
    """Value of the tensor product of block sparse grids (see the module
    docstring) for a product-form integrand."""
    from . import smolyak_factorised, smolyak_points
    if family == "corner_peak":
        raise ValueError("the corner-peak integrand does not factor over blocks")
    K = q - d
    if K < 0:
        raise ValueError("q < d")

    def block_value(db, bp):
        if method == "points":
            return smolyak_points(db, db + K, rule, family, bp)["q"]
        return smolyak_factorised(db, db + K, rule, family, bp)

    with mp.workdps(40):
        if family in ("oscillatory", "oscillatory_quadratic", "oscillatory_quadratic_linear"):
            z = mp.mpc(1)
            for s, ln in blocks(d, m):
                re = block_value(ln, block_params(family, params, d, s, ln, 0.0))
                im = block_value(ln, block_params(family, params, d, s, ln, -0.25))
                z *= mp.mpc(re, im)
            w = float(np.asarray(params, dtype=np.float64)[0])
            return float(mp.re(mp.expj(2 * mp.pi * mp.mpf(w)) * z))
        v = mp.mpf(1)
        for s, ln in blocks(d, m):
            v *= block_value(ln, block_params(family, params, d, s, ln))
        return float(v)
