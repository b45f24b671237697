"""CPU oracle for Smolyak sparse-grid quadrature -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it and
shares no code with it (no kernels, headers, helpers, tables or constants).

Contents
--------
* ``liboracle.so`` (built from ``sg_oracle.c``): 1-D rules of Section 2.2
  rebuilt from their formulas in binary128; canonical enumeration of the
  multi-index window of (2.6); the point-by-point Smolyak sum (2.6)-(2.7) in
  x87 extended precision; the factorised sum and its parameter gradient in
  binary128.
* ``counts``: exact integer counts of Section 2.1 (multi-indices in the window,
  the point count n_d^q with repetition, unique points), by enumeration and by
  generating functions, in Python integers.
* ``reference``: closed-form integrals of the test integrands.

Every function states the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "sg_oracle.c")

RULE_IDS = {"tr": 1, "cc": 2, "gp": 3, "gl": 4, "gl_paper": 5}
FAMILY_IDS = {"exp_sum": 0, "oscillatory": 1, "product_peak": 2, "monomial": 3, "corner_peak": 4,
              "gaussian": 5, "oscillatory_quadratic": 6, "oscillatory_quadratic_linear": 7}


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (no contraction of a*b+c into FMAs)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=gnu11", "-ffp-contract=off",
               "-Wall", "-Werror", "-Wno-unused-function", SRC_PATH, "-o", tmp,
               "-lquadmath", "-lpthread", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


SAN_LIB_PATH = os.path.join(_HERE, "liboracle_san.so")


def build_sanitized() -> str:
    """The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (for
    the CPU sanitizer tests; loaded in a process that preloads the runtimes)."""
    tmp = SAN_LIB_PATH + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O1", "-g", "-fPIC", "-shared", "-std=gnu11", "-ffp-contract=off", "-Wall", "-Werror",
           "-Wno-unused-function", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", SRC_PATH, "-o", tmp, "-lquadmath", "-lpthread", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, SAN_LIB_PATH)
    return SAN_LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = load(LIB_PATH)
    return _lib


def load(path: str):
    """Open an oracle library file and declare its functions."""
    if True:
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        L.or_rule_npoints.argtypes = [ctypes.c_int, ctypes.c_int]
        L.or_rule_npoints.restype = ctypes.c_long
        L.or_rule.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.or_rule.restype = ctypes.c_int
        L.or_enumerate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                   ctypes.c_int, ip, ip, ip]
        L.or_enumerate.restype = ctypes.c_uint64
        L.or_smolyak_points.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp,
                                        ctypes.c_int, ctypes.c_int, dp]
        L.or_smolyak_points.restype = ctypes.c_int
        L.or_smolyak_factorised.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            dp, dp]
        L.or_smolyak_factorised.restype = ctypes.c_int
        L.or_smolyak_factorised_grad.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                 ctypes.c_int, dp, dp]
        L.or_smolyak_factorised_grad.restype = ctypes.c_int
        L.or_batch_factorised.argtypes = [ctypes.c_int] + [ip] * 4 + [ctypes.POINTER(ctypes.c_int64), dp,
                                                                      ctypes.c_int, dp]
        L.or_batch_factorised.restype = ctypes.c_int
    return L


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def rule_npoints(rule: str, level: int) -> int:
    """n_l of Section 2.2 (level 1 is the single midpoint for every rule)."""
    return int(lib().or_rule_npoints(RULE_IDS[rule], level))


def rule(rule: str, level: int):
    """Level-l nodes and weights on [0,1] ((2.10), (2.11), (2.13)), ascending."""
    n = rule_npoints(rule, level)
    x = np.zeros(n)
    w = np.zeros(n)
    got = lib().or_rule(RULE_IDS[rule], level, _dp(x), _dp(w))
    if got != n:
        raise ValueError("bad rule/level")
    return x, w


def enumerate_window(d: int, q: int, start: int = 0, count: int | None = None, max_nnz: int | None = None):
    """Multi-indices of the window of (2.6) in canonical order.

    Order: by excess e = |l| - d ascending, then by (l_1..l_d) in decreasing
    lexicographic order.  Returns (total, coords, levels, nnz) where row r
    holds the sparse form (coordinates with l_i >= 2, ascending) of rank
    start + r.
    """
    K = q - d
    if max_nnz is None:
        max_nnz = max(1, K)
    L = lib()
    if count is None:
        total = int(L.or_enumerate(d, q, 0, 0, max_nnz, None, None, None))
        count = total - start
    coords = np.full((max(count, 1), max_nnz), -1, dtype=np.int32)
    levels = np.zeros((max(count, 1), max_nnz), dtype=np.int32)
    nnz = np.zeros(max(count, 1), dtype=np.int32)
    total = int(L.or_enumerate(d, q, start, count, max_nnz, _ip(coords), _ip(levels), _ip(nnz)))
    return total, coords[:count], levels[:count], nnz[:count]


def smolyak_points(d: int, q: int, rule: str, family: str, params, nthreads: int | None = None,
                   centred: bool = True) -> dict:
    """Point-by-point Smolyak sum (2.6)-(2.7) in extended precision.

    Returns dict(q=value, hi, lo, A=rounding scale, fc=f(centre), npoints).
    The rounding error is at most a small multiple of 2^-64 * (A + |fc|).
    """
    params = np.ascontiguousarray(params, dtype=np.float64)
    if nthreads is None:
        nthreads = min(16, os.cpu_count() or 1)
    out = np.zeros(5)
    rc = lib().or_smolyak_points(d, q, RULE_IDS[rule], FAMILY_IDS[family], _dp(params),
                                 nthreads, 1 if centred else 0, _dp(out))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    return dict(q=out[0] + out[1], hi=out[0], lo=out[1], A=out[2], fc=out[3], npoints=int(out[4]))


def smolyak_factorised(d: int, q: int, rule: str, family: str, params) -> float:
    """Factorised Smolyak sum (2.6) for product / exponential-ridge integrands,
    in binary128; returns the value rounded to double."""
    params = np.ascontiguousarray(params, dtype=np.float64)
    out = np.zeros(2)
    rc = lib().or_smolyak_factorised(d, q, RULE_IDS[rule], FAMILY_IDS[family], _dp(params), _dp(out))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    return float(out[0])


def smolyak_factorised_hilo(d: int, q: int, rule: str, family: str, params):
    params = np.ascontiguousarray(params, dtype=np.float64)
    out = np.zeros(2)
    rc = lib().or_smolyak_factorised(d, q, RULE_IDS[rule], FAMILY_IDS[family], _dp(params), _dp(out))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    return float(out[0]), float(out[1])


def smolyak_factorised_grad(d: int, q: int, rule: str, family: str, params) -> np.ndarray:
    """Gradient of the factorised sum with respect to every parameter."""
    params = np.ascontiguousarray(params, dtype=np.float64)
    g = np.zeros_like(params)
    rc = lib().or_smolyak_factorised_grad(d, q, RULE_IDS[rule], FAMILY_IDS[family], _dp(params), _dp(g))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    return g


def batch_factorised(batch, nthreads: int | None = None) -> np.ndarray:
    """Factorised value for every problem of a ``workloads.Batch`` (threaded
    over integrands; each value is exactly ``smolyak_factorised``'s)."""
    n = len(batch)
    if n == 0:
        return np.zeros(0)
    d = np.array([p.d for p in batch.problems], dtype=np.int32)
    q = np.array([p.q for p in batch.problems], dtype=np.int32)
    r = np.array([RULE_IDS[p.rule] for p in batch.problems], dtype=np.int32)
    f = np.array([FAMILY_IDS[p.family] for p in batch.problems], dtype=np.int32)
    off = np.array([p.param_offset for p in batch.problems], dtype=np.int64)
    params = np.ascontiguousarray(batch.params, dtype=np.float64)
    out = np.zeros(n)
    if nthreads is None:
        nthreads = min(16, os.cpu_count() or 1)
    rc = lib().or_batch_factorised(n, _ip(d), _ip(q), _ip(r), _ip(f),
                                   off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(params),
                                   nthreads, _dp(out))
    if rc != 0:
        raise ValueError("oracle rejected a problem")
    return out


def batch_points(batch, nthreads: int | None = None) -> np.ndarray:
    """Point-by-point value for every problem of a ``workloads.Batch``."""
    out = np.zeros(len(batch))
    for i, p in enumerate(batch.problems):
        out[i] = smolyak_points(p.d, p.q, p.rule, p.family, batch.param_slice(i), nthreads)["q"]
    return out


#: families of the form cos(2 pi w + phase(x)) with w the first parameter
OSCILLATORY_FAMILIES = ("oscillatory", "oscillatory_quadratic", "oscillatory_quadratic_linear")


class _ParamBatch:
    """Problems with a flat parameter array (the shape batch_factorised reads)."""

    def __init__(self, problems, params):
        self.problems = list(problems)
        self.params = params

    def __len__(self):
        return len(self.problems)


def quarter_shift(batch):
    """The batch with w replaced by w - 1/4 for every oscillatory integrand
    (same problems, a copy of the parameters).  Because the rule (2.6) is
    linear, Q(w) + i Q(w - 1/4) = e^{2 pi i w} S with S the Smolyak sum of
    the complex integrand e^{i phase(x)}: the shifted values are the
    imaginary parts of the complex rule."""
    params = np.array(batch.params, dtype=np.float64, copy=True)
    for p in batch.problems:
        if p.family in OSCILLATORY_FAMILIES:
            params[p.param_offset] -= 0.25
    return _ParamBatch(batch.problems, params)


def accuracy_scale(batch, ref, nthreads: int | None = None) -> np.ndarray:
    """Scale against which the error of each result is stated.

    Non-oscillatory families: |Q|.  Oscillatory families (the real part of
    e^{2 pi i w} S for a complex Smolyak sum S, see quarter_shift): the
    modulus |S| = sqrt(Q(w)^2 + Q(w - 1/4)^2), which does not depend on w.
    Q(w) itself passes through zero as w varies, so an error relative to
    |Q(w)| is unbounded near those zeros while the rule's rounding error is
    proportional to |S|.  ``ref`` holds the oracle's Q(w); the shifted values
    come from the binary128 factorised sum."""
    ref = np.asarray(ref, dtype=np.float64)
    osc = np.array([p.family in OSCILLATORY_FAMILIES for p in batch.problems])
    scale = np.abs(ref).copy()
    if osc.any():
        idx = np.nonzero(osc)[0]
        shifted = batch_factorised(quarter_shift(_ParamBatch([batch.problems[i] for i in idx], batch.params)),
                                   nthreads)
        scale[idx] = np.hypot(ref[idx], shifted)
    return scale


def accuracy_scale_one(d: int, q: int, rule: str, family: str, params, ref: float) -> float:
    """accuracy_scale for one integrand."""
    if family not in OSCILLATORY_FAMILIES:
        return abs(ref)
    sp = np.array(params, dtype=np.float64, copy=True)
    sp[0] -= 0.25
    return float(np.hypot(ref, smolyak_factorised(d, q, rule, family, sp)))


from . import counts, reference  # noqa: E402,F401
