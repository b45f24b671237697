"""Closed-form integrals of the test integrands -- TEST INFRASTRUCTURE ONLY.

I_d(f) of (2.1), on the unit cube, for the test families, in mpmath at 40
significant digits.  These are the exact integrals, not the Smolyak values:
they pin the quadrature only where its truncation error is small.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np

mp.mp.dps = 40


def exact_exp_sum(c) -> float:
    """prod_i (e^{c_i} - 1)/c_i  (factor 1 when c_i = 0)."""
    r = mp.mpf(1)
    for ci in np.asarray(c, dtype=np.float64):
        ci = mp.mpf(float(ci))
        r *= mp.expm1(ci) / ci if ci != 0 else mp.mpf(1)
    return r


def exact_oscillatory(w, a):
    """Re( e^{2 pi i w} prod_i (e^{i a_i} - 1)/(i a_i) )."""
    z = mp.expj(2 * mp.pi * mp.mpf(float(w)))
    for ai in np.asarray(a, dtype=np.float64):
        ai = mp.mpf(float(ai))
        z *= (mp.expj(ai) - 1) / (1j * ai) if ai != 0 else mp.mpf(1)
    return mp.re(z)


def exact_product_peak(b, u):
    """prod_i b_i (atan(b_i (1-u_i)) + atan(b_i u_i))."""
    r = mp.mpf(1)
    for bi, ui in zip(np.asarray(b, dtype=np.float64), np.asarray(u, dtype=np.float64)):
        bi = mp.mpf(float(bi))
        ui = mp.mpf(float(ui))
        r *= bi * (mp.atan(bi * (1 - ui)) + mp.atan(bi * ui))
    return r


def exact_corner_peak(a):
    """Integral of (1 + sum a_i x_i)^-(d+1) over [0,1]^d for a_i > 0: by d
    successive integrations, (1 / (d! prod a_i)) sum over subsets S of
    (-1)^|S| / (1 + sum_{i in S} a_i).  The alternating sum cancels heavily,
    so it is evaluated at the working precision raised with d."""
    a = [float(x) for x in np.asarray(a, dtype=np.float64)]
    d = len(a)
    with mp.workdps(40 + 4 * d):
        am = [mp.mpf(x) for x in a]
        tot = mp.mpf(0)
        for mask in range(1 << d):
            s = mp.mpf(1)
            bits = 0
            for i in range(d):
                if mask >> i & 1:
                    s += am[i]
                    bits += 1
            tot += (-1) ** bits / s
        r = tot / (mp.factorial(d) * mp.fprod(am))
        return +r


def _quad_exp_1d(k, u):
    """int_0^1 exp(k (x - u)^2) dx for real or complex k: with s = x - u and
    r = sqrt(-k), (sqrt(pi) / (2 r)) (erf(r (1 - u)) + erf(r u))."""
    k = mp.mpc(k)
    u = mp.mpf(float(u))
    if k == 0:
        return mp.mpf(1)
    r = mp.sqrt(-k)
    return mp.sqrt(mp.pi) / (2 * r) * (mp.erf(r * (1 - u)) + mp.erf(r * u))


def exact_gaussian(c, u):
    """prod_i int_0^1 exp(c_i (x - u_i)^2) dx (real part: the integral is real)."""
    r = mp.mpc(1)
    for ci, ui in zip(np.asarray(c, dtype=np.float64), np.asarray(u, dtype=np.float64)):
        r *= _quad_exp_1d(mp.mpf(float(ci)), ui)
    return mp.re(r)


def exact_oscillatory_quadratic(w, a, u):
    """Re( e^{2 pi i w} prod_i int_0^1 exp(i a_i (x - u_i)^2) dx )."""
    z = mp.expj(2 * mp.pi * mp.mpf(float(w)))
    for ai, ui in zip(np.asarray(a, dtype=np.float64), np.asarray(u, dtype=np.float64)):
        z *= _quad_exp_1d(1j * mp.mpf(float(ai)), ui)
    return mp.re(z)


def _quad_linear_1d(a, u, c):
    """int_0^1 exp(i (a (x - u)^2 + c x)) dx.  a != 0: completing the square,
    a (x - u)^2 + c x = a (x - v)^2 + c u - c^2 / (4 a) with v = u - c / (2 a),
    so the integral is e^{i (c u - c^2/(4a))} times _quad_exp_1d(i a, v) (the
    error functions at 40 + digits, with the working precision raised by
    the decimal size of v); a = 0: (e^{i c} - 1) / (i c), or 1 at c = 0."""
    a = mp.mpf(float(a))
    u = mp.mpf(float(u))
    c = mp.mpf(float(c))
    if a == 0:
        return mp.mpf(1) if c == 0 else (mp.expj(c) - 1) / (1j * c)
    v = u - c / (2 * a)
    extra = int(max(0, mp.log10(abs(v) + 1))) * 2 + 10
    with mp.workdps(mp.mp.dps + extra):
        k = 1j * a
        r = mp.sqrt(-k)
        base = mp.sqrt(mp.pi) / (2 * r) * (mp.erf(r * (1 - v)) + mp.erf(r * v))
        val = mp.expj(c * u - c * c / (4 * a)) * base
    return +val


def exact_oscillatory_quadratic_linear(w, a, u, c):
    """Re( e^{2 pi i w} prod_i int_0^1 exp(i (a_i (x - u_i)^2 + c_i x)) dx )."""
    z = mp.expj(2 * mp.pi * mp.mpf(float(w)))
    for ai, ui, ci in zip(np.asarray(a, dtype=np.float64), np.asarray(u, dtype=np.float64),
                          np.asarray(c, dtype=np.float64)):
        z *= _quad_linear_1d(ai, ui, ci)
    return mp.re(z)


def exact(family: str, d: int, params):
    params = np.asarray(params, dtype=np.float64)
    if family == "corner_peak":
        return exact_corner_peak(params[:d])
    if family == "exp_sum":
        return exact_exp_sum(params[:d])
    if family == "oscillatory":
        return exact_oscillatory(params[0], params[1:1 + d])
    if family == "product_peak":
        return exact_product_peak(params[:d], params[d:2 * d])
    if family == "gaussian":
        return exact_gaussian(params[:d], params[d:2 * d])
    if family == "oscillatory_quadratic":
        return exact_oscillatory_quadratic(params[0], params[1:1 + d], params[1 + d:1 + 2 * d])
    if family == "oscillatory_quadratic_linear":
        return exact_oscillatory_quadratic_linear(params[0], params[1:1 + d], params[1 + d:1 + 2 * d],
                                                  params[1 + 2 * d:1 + 3 * d])
    raise ValueError(family)


def exact_grad_oscillatory(w, a) -> np.ndarray:
    """Gradient of the exact oscillatory integral with respect to (w, a)."""
    a = [mp.mpf(float(x)) for x in np.asarray(a, dtype=np.float64)]
    rot = mp.expj(2 * mp.pi * mp.mpf(float(w)))
    facs = [(mp.expj(ai) - 1) / (1j * ai) for ai in a]
    dfacs = []
    for ai in a:
        # d/da (e^{ia}-1)/(ia) = (i a e^{ia} i - i (e^{ia} - 1)) / (i a)^2 ... written out:
        # g(a) = (e^{ia} - 1)/(ia);  g'(a) = e^{ia}/a - (e^{ia} - 1)/(i a^2)
        dfacs.append(mp.expj(ai) / ai - (mp.expj(ai) - 1) / (1j * ai * ai))
    total = rot
    for f in facs:
        total *= f
    g = np.zeros(len(a) + 1)
    g[0] = float(mp.re(2j * mp.pi * total))
    for t in range(len(a)):
        z = rot * dfacs[t]
        for s, f in enumerate(facs):
            if s != t:
                z *= f
        g[1 + t] = float(mp.re(z))
    return g
