"""Seeded synthetic workloads: integrand batches and their parameters.

This module only draws random inputs.  It holds none of the quadrature's
arithmetic (no rules, no counts, no sums), so that the GPU path and the CPU
oracle can both be fed from it without sharing any part of the method.

Integrand families (all on the unit cube [0,1]^d, a rescaling of the paper's
[-1,1]^d in (2.1)):

* ``exp_sum``      f(x) = exp(sum_i c_i x_i)            params: c[d]
* ``oscillatory``  f(x) = cos(2 pi w + sum_i a_i x_i)    params: w, a[d]
* ``product_peak`` f(x) = prod_i 1/(b_i^-2 + (x_i-u_i)^2) params: b[d], u[d]

The product-peak family is the integrand of Test 4 (4.4) and Table 5.8 with
free widths and centres; exp-sum generalises (4.5)/(5.1); oscillatory
generalises the cosine integrand of Table 5.7.

A batch is a list of problems ``(d, q, rule, family, param_offset)`` plus one
flat float64 parameter array.  Rules are named ``"cc"`` (Clenshaw-Curtis,
(2.11)), ``"tr"`` (trapezoidal, (2.10)), ``"gl"`` (Gauss-Legendre with 2l-1
points at level l) and ``"gl_paper"`` (Gauss-Legendre with l points at level
l, (2.13)).  The level q is the q of (2.6); the excess budget is K = q - d.

Random numbers come from ``numpy.random.default_rng(seed)`` (PCG64) and are
drawn per integrand in a fixed order: shape choices first, then the scalar
parameter (w), then the vectors in coordinate order (a; or b then u; or c).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np

RULES = ("tr", "cc", "gl", "gl_paper")
# every rule a problem may name; the default mixes above keep the four
# original rules so that seeded workloads do not change
ALL_RULES = RULES + ("gp",)
#: families the factorised sweep handles (they factor per coordinate)
FAMILIES = ("exp_sum", "oscillatory", "product_peak")
#: families only the point-by-point path handles (ridge functions that do not factor)
POINT_ONLY_FAMILIES = ("corner_peak",)
#: families the sweep handles beyond FAMILIES (kept out of the default mixes;
#: the oscillatory quadratics on the complex sweep)
EXTRA_SWEEP_FAMILIES = ("gaussian", "oscillatory_quadratic", "oscillatory_quadratic_linear")

#: seeds used for the five standard workloads (workload k uses SEED_BASE + k)
SEED_BASE = 14313


def n_params(family: str, d: int) -> int:
    """Number of float64 parameters one integrand of ``family`` takes."""
    if family == "exp_sum":
        return d
    if family == "oscillatory":
        return d + 1
    if family == "product_peak":
        return 2 * d
    if family == "corner_peak":
        return d
    if family == "gaussian":
        return 2 * d
    if family == "oscillatory_quadratic":
        return 2 * d + 1
    if family == "oscillatory_quadratic_linear":
        return 3 * d + 1
    raise ValueError(f"unknown family {family!r}")


@dataclass
class Problem:
    d: int
    q: int
    rule: str
    family: str
    param_offset: int

    @property
    def K(self) -> int:
        return self.q - self.d


@dataclass
class Batch:
    """A batch of integrands sharing one flat parameter array."""

    name: str
    problems: List[Problem] = field(default_factory=list)
    params: np.ndarray = field(default_factory=lambda: np.zeros(0))

    def __len__(self) -> int:
        return len(self.problems)

    def param_slice(self, i: int) -> np.ndarray:
        p = self.problems[i]
        return self.params[p.param_offset:p.param_offset + n_params(p.family, p.d)]

    def subset(self, idx: Sequence[int], name: str | None = None) -> "Batch":
        """A new batch holding problems ``idx`` with compacted parameters."""
        probs, chunks, off = [], [], 0
        for i in idx:
            p = self.problems[i]
            v = self.param_slice(i)
            probs.append(Problem(p.d, p.q, p.rule, p.family, off))
            chunks.append(v)
            off += len(v)
        params = np.concatenate(chunks) if chunks else np.zeros(0)
        return Batch(name or f"{self.name}[subset]", probs, params.astype(np.float64))


class _Builder:
    def __init__(self, name: str):
        self.name = name
        self.problems: List[Problem] = []
        self.chunks: List[np.ndarray] = []
        self.off = 0

    def add(self, d: int, q: int, rule: str, family: str, params: np.ndarray):
        assert rule in ALL_RULES and (family in FAMILIES or family in POINT_ONLY_FAMILIES
                                      or family in EXTRA_SWEEP_FAMILIES)
        params = np.asarray(params, dtype=np.float64).ravel()
        assert params.size == n_params(family, d)
        self.problems.append(Problem(int(d), int(q), rule, family, self.off))
        self.chunks.append(params)
        self.off += params.size

    def build(self) -> Batch:
        params = np.concatenate(self.chunks) if self.chunks else np.zeros(0)
        return Batch(self.name, self.problems, params.astype(np.float64))


def draw_params(rng: np.random.Generator, family: str, d: int,
                osc_scale: float = 9.0, exp_scale: float = 1.0) -> np.ndarray:
    """Draw one integrand's parameters with the standard distributions.

    exp_sum: c_i ~ U(0,1) * exp_scale.  oscillatory: w ~ U(0,1),
    a_i ~ U(0,1) * osc_scale / d.  product_peak: b_i ~ U(0.5, 2),
    u_i ~ U(0, 1).  corner_peak: a_i ~ U(0,1), normalised to sum 1.
    gaussian: c_i ~ U(-4, 2) * 4 / d, u_i ~ U(0, 1).  oscillatory_quadratic:
    w ~ U(0,1), a_i ~ U(-1, 1) * osc_scale / d, u_i ~ U(0, 1).
    oscillatory_quadratic_linear: the same, then c_i ~ U(-1, 1) * osc_scale / d.
    """
    if family == "exp_sum":
        return rng.uniform(0.0, 1.0, d) * exp_scale
    if family == "oscillatory":
        w = rng.uniform(0.0, 1.0)
        a = rng.uniform(0.0, 1.0, d) * (osc_scale / d)
        return np.concatenate([[w], a])
    if family == "product_peak":
        b = rng.uniform(0.5, 2.0, d)
        u = rng.uniform(0.0, 1.0, d)
        return np.concatenate([b, u])
    if family == "corner_peak":
        # a_i ~ U(0,1) scaled so that sum a_i = 1 (a mild corner)
        a = rng.uniform(0.0, 1.0, d)
        return a / a.sum()
    if family == "gaussian":
        c = rng.uniform(-4.0, 2.0, d) * (4.0 / d)
        u = rng.uniform(0.0, 1.0, d)
        return np.concatenate([c, u])
    if family == "oscillatory_quadratic":
        w = rng.uniform(0.0, 1.0)
        a = rng.uniform(-1.0, 1.0, d) * (osc_scale / d)
        u = rng.uniform(0.0, 1.0, d)
        return np.concatenate([[w], a, u])
    if family == "oscillatory_quadratic_linear":
        w = rng.uniform(0.0, 1.0)
        a = rng.uniform(-1.0, 1.0, d) * (osc_scale / d)
        u = rng.uniform(0.0, 1.0, d)
        c = rng.uniform(-1.0, 1.0, d) * (osc_scale / d)
        return np.concatenate([[w], a, u, c])
    raise ValueError(family)


def plain_exp_d10(seed: int = SEED_BASE + 1) -> Batch:
    """One exp-sum integrand, d=10, q=d+4, Clenshaw-Curtis, c_i ~ U(0,1)."""
    rng = np.random.default_rng(seed)
    b = _Builder("plain_exp_d10_q14_cc")
    b.add(10, 14, "cc", "exp_sum", rng.uniform(0.0, 1.0, 10))
    return b.build()


def precision_d100(seed: int = SEED_BASE + 2) -> Batch:
    """d=100, q=d+5, Clenshaw-Curtis: one oscillatory (w ~ U(0,1),
    a_i ~ U(0,1)*9/d) and one product-peak (b_i ~ U(0.5,2), u_i ~ U(0,1))."""
    rng = np.random.default_rng(seed)
    b = _Builder("precision_d100_q105_cc")
    d = 100
    b.add(d, d + 5, "cc", "oscillatory", draw_params(rng, "oscillatory", d))
    b.add(d, d + 5, "cc", "product_peak", draw_params(rng, "product_peak", d))
    return b.build()


def high_dim_d1000(seed: int = SEED_BASE + 3, rules: Sequence[str] = ("gl", "tr")) -> Batch:
    """d=1000, q=d+3: exp(sum c_i x_i / d) with c_i ~ U(-1,1), once per rule.

    The same c vector is used for every rule; the parameter passed to the
    exp-sum family is c_i / d.
    """
    rng = np.random.default_rng(seed)
    d = 1000
    c = rng.uniform(-1.0, 1.0, d) / d
    b = _Builder("high_dim_d1000_q1003")
    for r in rules:
        b.add(d, d + 3, r, "exp_sum", c)
    return b.build()


def batched_uneven(n: int = 4096, seed: int = SEED_BASE + 4,
                   d_lo: int = 8, d_hi: int = 256, k_lo: int = 2, k_hi: int = 6,
                   rules: Sequence[str] = ("cc", "gl"),
                   families: Sequence[str] = ("oscillatory", "exp_sum")) -> Batch:
    """Batch of ``n`` integrands of uneven size.

    Per integrand, in this order: d ~ U{d_lo..d_hi}, K = q-d ~ U{k_lo..k_hi},
    rule uniform over ``rules``, family uniform over ``families``, then the
    parameters (exp-sum c_i ~ U(0,1); oscillatory w ~ U(0,1),
    a_i ~ U(0,1)*9/d).
    """
    rng = np.random.default_rng(seed)
    b = _Builder(f"batched_uneven_n{n}")
    for _ in range(n):
        d = int(rng.integers(d_lo, d_hi + 1))
        K = int(rng.integers(k_lo, k_hi + 1))
        rule = rules[int(rng.integers(0, len(rules)))]
        fam = families[int(rng.integers(0, len(families)))]
        b.add(d, d + K, rule, fam, draw_params(rng, fam, d))
    return b.build()


def gradient_osc_d200(n: int = 256, seed: int = SEED_BASE + 5, d: int = 200, K: int = 5) -> Batch:
    """``n`` oscillatory integrands, d=200, q=d+5, Clenshaw-Curtis."""
    rng = np.random.default_rng(seed)
    b = _Builder(f"gradient_osc_d{d}_n{n}")
    for _ in range(n):
        b.add(d, d + K, "cc", "oscillatory", draw_params(rng, "oscillatory", d))
    return b.build()


def oscillatory_quadratic_d1000(seed: int = SEED_BASE + 10, d: int = 1000, K: int = 4, rule: str = "gp") -> Batch:
    """One oscillatory-quadratic integrand cos(2 pi w + sum a_i (x_i - u_i)^2)
    (the sines of (4.1)/(4.2) in d dimensions), q = d + K, standard draws."""
    rng = np.random.default_rng(seed)
    return single(d, d + K, rule, "oscillatory_quadratic", draw_params(rng, "oscillatory_quadratic", d))


def random_small(seed: int, n: int, d_range=(1, 6), k_range=(0, 4),
                 rules: Sequence[str] = RULES, families: Sequence[str] = FAMILIES,
                 osc_scale: float = 9.0, exp_scale: float = 1.0) -> Batch:
    """Small mixed batch for parity tests (sizes the point oracle finishes fast)."""
    rng = np.random.default_rng(seed)
    b = _Builder(f"random_small_s{seed}")
    for _ in range(n):
        d = int(rng.integers(d_range[0], d_range[1] + 1))
        K = int(rng.integers(k_range[0], k_range[1] + 1))
        rule = rules[int(rng.integers(0, len(rules)))]
        fam = families[int(rng.integers(0, len(families)))]
        b.add(d, d + K, rule, fam, draw_params(rng, fam, d, osc_scale, exp_scale))
    return b.build()


def single(d: int, q: int, rule: str, family: str, params) -> Batch:
    """A one-integrand batch with explicit parameters."""
    b = _Builder(f"single_{family}_{rule}_d{d}_q{q}")
    b.add(d, q, rule, family, np.asarray(params, dtype=np.float64))
    return b.build()


def concat(batches: Sequence[Batch], name: str = "concat") -> Batch:
    b = _Builder(name)
    for bt in batches:
        for i, p in enumerate(bt.problems):
            b.add(p.d, p.q, p.rule, p.family, bt.param_slice(i))
    return b.build()


STANDARD = {
    "plain_exp_d10": plain_exp_d10,
    "precision_d100": precision_d100,
    "high_dim_d1000": high_dim_d1000,
    "batched_uneven": batched_uneven,
    "gradient_osc_d200": gradient_osc_d200,
}
