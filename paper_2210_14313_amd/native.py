"""ctypes binding of libsgmdi.so (include/sgmdi.h): argument marshalling only.

Every step of the computation runs in the library's HIP kernels; this module
converts Python/torch objects to pointers and sizes and raises on errors.
It never falls back to another implementation: if the library is missing,
loading fails with an exception.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SGMDI_LIB: developer override of the library file (kernel variants)
LIB_PATH = os.environ.get("SGMDI_LIB") or os.path.join(_HERE, "libsgmdi.so")

RULES = {"tr": 1, "cc": 2, "gp": 3, "gl": 4, "gl_paper": 5}
FAMILIES = {"exp_sum": 0, "oscillatory": 1, "product_peak": 2, "corner_peak": 3, "gaussian": 4,
            "oscillatory_quadratic": 5, "oscillatory_quadratic_linear": 6}
PRECISIONS = {"fp64": 0, "fp32c": 1, "fp32e": 2}
STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "overflow", 4: "out of memory",
          5: "device error", 6: "capture error"}
MAX_K = 8


class SgError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        super().__init__(f"sgmdi: {STATUS.get(status, status)}{': ' + msg if msg else ''}")
        self.status = status


class SgProblem(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("q", ctypes.c_int32), ("rule", ctypes.c_int32),
                ("family", ctypes.c_int32), ("param_offset", ctypes.c_int64)]


class SgPlanInfo(ctypes.Structure):
    _fields_ = [("effective_points", ctypes.c_uint64), ("units", ctypes.c_uint64),
                ("pair_evals", ctypes.c_uint64), ("macs", ctypes.c_uint64),
                ("merge_flops", ctypes.c_uint64), ("block_threads", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("coords_per_lane", ctypes.c_int32),
                ("max_group", ctypes.c_int32), ("graph", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("cost_scaled", ctypes.c_int32), ("balanced", ctypes.c_int32),
                ("fp64_complex", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None

EXPORTS = ["sg_context_create", "sg_context_destroy", "sg_status_string", "sg_last_error", "sg_counts",
           "sg_rule_table", "sg_coefficient", "sg_unrank", "sg_unrank_device", "sg_plan_create",
           "sg_plan_execute", "sg_plan_execute_grad", "sg_plan_get_info", "sg_plan_autotune",
           "sg_plan_set_schedule", "sg_plan_set_schedule_balanced", "sg_plan_destroy", "sg_integrate",
           "sg_integrate_noalloc", "sg_integrate_points", "sg_plan_create_blocked", "sg_version",
           "sg_context_save_tuning", "sg_context_load_tuning"]


def lib():
    """Load libsgmdi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2210_14313_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, u64, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64
    P = ctypes.POINTER
    sig = {
        "sg_context_create": ([P(vp)], i32),
        "sg_context_destroy": ([vp], i32),
        "sg_status_string": ([i32], ctypes.c_char_p),
        "sg_last_error": ([vp], ctypes.c_char_p),
        "sg_counts": ([i32, i32, i32, P(u64), P(u64), P(u64)], i32),
        "sg_rule_table": ([i32, i32, P(ctypes.c_double), P(ctypes.c_double), P(i32)], i32),
        "sg_coefficient": ([i32, i32, i32, P(i64)], i32),
        "sg_unrank": ([i32, i32, u64, P(i32), P(i32), P(i32)], i32),
        "sg_unrank_device": ([vp, i32, i32, u64, u64, i32, vp, vp, vp, vp], i32),
        "sg_plan_create": ([vp, P(SgProblem), i32, i32, P(vp)], i32),
        "sg_plan_create_blocked": ([vp, P(SgProblem), i32, i32, i32, P(vp)], i32),
        "sg_plan_execute": ([vp, vp, vp, vp, vp], i32),
        "sg_plan_execute_grad": ([vp, vp, vp, vp, vp], i32),
        "sg_plan_get_info": ([vp, P(SgPlanInfo)], i32),
        "sg_plan_autotune": ([vp, vp, vp, vp], i32),
        "sg_plan_set_schedule": ([vp, i32, i32, i32, i32, i32], i32),
        "sg_plan_set_schedule_balanced": ([vp, i32, i32], i32),
        "sg_plan_destroy": ([vp], i32),
        "sg_integrate": ([vp, P(SgProblem), i32, vp, vp, vp, vp], i32),
        "sg_integrate_noalloc": ([vp, P(SgProblem), i32, vp, vp, vp, vp], i32),
        "sg_integrate_points": ([vp, P(SgProblem), vp, vp, vp, u64, vp], i32),
        "sg_version": ([], ctypes.c_char_p),
        "sg_context_save_tuning": ([vp, ctypes.c_char_p], i32),
        "sg_context_load_tuning": ([vp, ctypes.c_char_p, P(i32)], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(st: int, ctx=None):
    if st != 0:
        msg = ""
        if ctx is not None and getattr(ctx, "value", None):
            msg = lib().sg_last_error(ctx).decode(errors="replace")
        raise SgError(st, msg)


# ------------------------------------------------------------- host calls
def version() -> str:
    return lib().sg_version().decode()


def counts(d: int, q: int, rule: str):
    """(n_multi, n_points_rep, n_points_unique) of the window of (2.6)."""
    a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib().sg_counts(d, q, RULES[rule], ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def rule_table(rule: str, level: int):
    n = ctypes.c_int32()
    _check(lib().sg_rule_table(RULES[rule], level, None, None, ctypes.byref(n)))
    x = np.zeros(n.value)
    w = np.zeros(n.value)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib().sg_rule_table(RULES[rule], level, x.ctypes.data_as(dp), w.ctypes.data_as(dp), ctypes.byref(n)))
    return x, w


def coefficient(d: int, q: int, e: int) -> int:
    c = ctypes.c_int64()
    _check(lib().sg_coefficient(d, q, e, ctypes.byref(c)))
    return c.value


def unrank(d: int, q: int, rank: int):
    K = max(1, q - d)
    co = (ctypes.c_int32 * K)()
    le = (ctypes.c_int32 * K)()
    nnz = ctypes.c_int32()
    _check(lib().sg_unrank(d, q, rank, co, le, ctypes.byref(nnz)))
    return [(co[i], le[i]) for i in range(nnz.value)]


# ------------------------------------------------------------- device side
def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Context:
    """Owns an sg_context on the current device."""

    def __init__(self):
        self.handle = ctypes.c_void_p()
        _check(lib().sg_context_create(ctypes.byref(self.handle)))

    def close(self):
        if self.handle:
            lib().sg_context_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def save_tuning(self, path: str) -> None:
        """Write the context's autotune results (sg_context_save_tuning)."""
        _check(lib().sg_context_save_tuning(self.handle, os.fsencode(path)), self.handle)

    def load_tuning(self, path: str) -> int:
        """Read autotune results; returns how many records were loaded (0 for
        a file of another library version or device)."""
        n = ctypes.c_int32(0)
        _check(lib().sg_context_load_tuning(self.handle, os.fsencode(path), ctypes.byref(n)), self.handle)
        return n.value

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx: Optional[Context] = None


def default_context() -> Context:
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context()
    return _default_ctx


def make_problems(problems) -> ctypes.Array:
    """sg_problem array from objects with d, q, rule, family, param_offset."""
    arr = (SgProblem * len(problems))()
    for i, p in enumerate(problems):
        arr[i] = SgProblem(p.d, p.q, RULES[p.rule], FAMILIES[p.family], p.param_offset)
    return arr


# Parameters of one integrand by family (include/sgmdi.h, sg_family).
_PARAMS_PER_FAMILY = {"exp_sum": (1, 0), "oscillatory": (1, 1), "product_peak": (2, 0), "corner_peak": (1, 0),
                      "gaussian": (2, 0), "oscillatory_quadratic": (2, 1), "oscillatory_quadratic_linear": (3, 1)}


def n_params(family: str, d: int) -> int:
    a, b = _PARAMS_PER_FAMILY[family]
    return a * d + b


def param_extent(problems: Sequence) -> int:
    """Elements of the parameter array the problems read: the largest
    param_offset + n_params(family, d)."""
    return max((int(p.param_offset) + n_params(p.family, p.d) for p in problems), default=0)


def check_tensor(name: str, t, min_numel: int):
    """The C ABI takes raw pointers it cannot bound: every tensor handed to it
    must be a contiguous float64 device tensor of at least min_numel
    elements (ValueError otherwise, before anything is launched)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 device tensor")
    if t.numel() < min_numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs >= {min_numel}")


class Plan:
    """A compiled batch: sg_plan_create / execute / execute_grad / destroy."""

    def __init__(self, problems: Sequence, precision: str = "fp64", ctx: Optional[Context] = None,
                 block_dims: int = 0):
        """block_dims > 0: the block (tensor-product) variant of the rule,
        sg_plan_create_blocked, with blocks of that many coordinates."""
        self.ctx = ctx or default_context()
        self.n = len(problems)
        self.problems = list(problems)
        self._arr = make_problems(problems)
        self.handle = ctypes.c_void_p()
        self.precision = precision
        self.param_extent = param_extent(self.problems)
        self.block_dims = int(block_dims)
        if self.block_dims > 0:
            _check(lib().sg_plan_create_blocked(self.ctx.handle, self._arr, self.n, PRECISIONS[precision],
                                                self.block_dims, ctypes.byref(self.handle)), self.ctx.handle)
        else:
            _check(lib().sg_plan_create(self.ctx.handle, self._arr, self.n, PRECISIONS[precision],
                                        ctypes.byref(self.handle)), self.ctx.handle)
        self._exec = lib().sg_plan_execute

    def info(self) -> dict:
        inf = SgPlanInfo()
        _check(lib().sg_plan_get_info(self.handle, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in SgPlanInfo._fields_}

    def execute(self, params, out=None, bound=None, stream=None):
        import torch
        check_tensor("params", params, self.param_extent)
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device=params.device)
        check_tensor("out", out, self.n)
        bptr = None
        if bound is not None:
            check_tensor("bound", bound, self.n)
            bptr = bound.data_ptr()
        st = self._exec(self.handle, params.data_ptr(), out.data_ptr(), bptr, _stream_ptr(stream))
        if st != 0:
            _check(st, self.ctx.handle)
        return out

    def execute_raw(self, params_ptr: int, out_ptr: int, bound_ptr: Optional[int] = None, stream=None):
        """sg_plan_execute on raw device-accessible addresses (e.g. the device
        alias of pinned host memory for the result)."""
        st = self._exec(self.handle, params_ptr, out_ptr, bound_ptr, _stream_ptr(stream))
        if st != 0:
            _check(st, self.ctx.handle)

    def execute_grad(self, params, grad_out, grad_params=None, stream=None):
        import torch
        check_tensor("params", params, self.param_extent)
        check_tensor("grad_out", grad_out, self.n)
        if grad_params is None:
            grad_params = torch.zeros_like(params)
        check_tensor("grad_params", grad_params, self.param_extent)
        _check(lib().sg_plan_execute_grad(self.handle, _ptr(params), _ptr(grad_out), _ptr(grad_params),
                                          _stream_ptr(stream)), self.ctx.handle)
        return grad_params

    def autotune(self, params, out, stream=None):
        check_tensor("params", params, self.param_extent)
        check_tensor("out", out, self.n)
        _check(lib().sg_plan_autotune(self.handle, _ptr(params), _ptr(out), _stream_ptr(stream)), self.ctx.handle)

    def set_schedule(self, coords_per_lane: int, max_group: int, graph: bool = False, persistent: bool = False,
                     cost_scaled: bool = False):
        _check(lib().sg_plan_set_schedule(self.handle, coords_per_lane, max_group, int(cost_scaled), int(persistent),
                                          int(graph)), self.ctx.handle)

    def set_balanced(self, waves_per_simd: int, graph: bool = False):
        """Balanced forward schedule (sg_plan_set_schedule_balanced)."""
        _check(lib().sg_plan_set_schedule_balanced(self.handle, int(waves_per_simd), int(graph)), self.ctx.handle)

    def close(self):
        if self.handle:
            lib().sg_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def integrate_one(problem, params, precision: str = "fp64", out=None, bound=None, stream=None,
                  ctx: Optional[Context] = None):
    """Plain single-integrand path (one launch, no plan, no graph)."""
    import torch
    check_tensor("params", params, n_params(problem.family, problem.d))
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=params.device)
    check_tensor("out", out, 1)
    if bound is not None:
        check_tensor("bound", bound, 1)
    ctx = ctx or default_context()
    pr = SgProblem(problem.d, problem.q, RULES[problem.rule], FAMILIES[problem.family], 0)
    _check(lib().sg_integrate(ctx.handle, ctypes.byref(pr), PRECISIONS[precision], _ptr(params), _ptr(out),
                              _ptr(bound), _stream_ptr(stream)), ctx.handle)
    return out


def integrate_noalloc(problem, params, precision: str = "fp64", out=None, bound=None, stream=None,
                      ctx: Optional[Context] = None):
    """The plan-free path without device allocation (sg_integrate_noalloc):
    out (and bound) must be given, so nothing is allocated here either."""
    if out is None:
        raise ValueError("integrate_noalloc needs an out tensor (it allocates nothing)")
    check_tensor("params", params, n_params(problem.family, problem.d))
    check_tensor("out", out, 1)
    if bound is not None:
        check_tensor("bound", bound, 1)
    ctx = ctx or default_context()
    pr = SgProblem(problem.d, problem.q, RULES[problem.rule], FAMILIES[problem.family], 0)
    _check(lib().sg_integrate_noalloc(ctx.handle, ctypes.byref(pr), PRECISIONS[precision], _ptr(params), _ptr(out),
                                      _ptr(bound), _stream_ptr(stream)), ctx.handle)
    return out


def integrate_points(problem, params, out=None, bound=None, max_points: int = 0, stream=None,
                     ctx: Optional[Context] = None):
    """Literal point-by-point path (sg_integrate_points): one integrand, FP64."""
    import torch
    check_tensor("params", params, n_params(problem.family, problem.d))
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=params.device)
    check_tensor("out", out, 1)
    if bound is not None:
        check_tensor("bound", bound, 1)
    ctx = ctx or default_context()
    pr = SgProblem(problem.d, problem.q, RULES[problem.rule], FAMILIES[problem.family], 0)
    _check(lib().sg_integrate_points(ctx.handle, ctypes.byref(pr), _ptr(params), _ptr(out), _ptr(bound),
                                     max_points, _stream_ptr(stream)), ctx.handle)
    return out


def unrank_device(d: int, q: int, rank0: int, count: int, max_nnz: Optional[int] = None, stream=None,
                  ctx: Optional[Context] = None):
    import torch
    ctx = ctx or default_context()
    K = q - d
    max_nnz = max_nnz or max(1, K)
    coords = torch.empty((max(count, 1), max_nnz), dtype=torch.int32, device="cuda")
    levels = torch.empty_like(coords)
    nnz = torch.empty(max(count, 1), dtype=torch.int32, device="cuda")
    _check(lib().sg_unrank_device(ctx.handle, d, q, rank0, count, max_nnz, _ptr(coords), _ptr(levels), _ptr(nnz),
                                  _stream_ptr(stream)), ctx.handle)
    return coords[:count], levels[:count], nnz[:count]
