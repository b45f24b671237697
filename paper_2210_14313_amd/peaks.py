"""ctypes binding of libsgpeaks.so (include/sgpeaks.h) and the measurement
of per-operation VALU ceilings on the current device.

measure() launches each probe kernel on a stream, times the launches with
HIP events on that stream, and returns operations per second per class.
The ceilings feed the serial-issue roofline of the dimension sweep:
T_min = sum over operation classes of n_op / peak_op.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsgpeaks.so")

OPS = {"v_fmac_f32": 0, "v_fma_f32": 1, "v_add_f32": 2, "v_fmac_f64": 3, "v_fma_f64": 4, "v_add_f64": 5,
       "v_exp_f32": 6, "v_sin_f32": 7, "v_cos_f32": 8, "v_rcp_f32": 9, "v_log_f32": 10, "v_rcp_f64": 11,
       "v_exp_f32+v_fmac_f32": 12}
EXPORTS = ["sgp_launch", "sgp_op_name"]

_lib = None


def lib():
    """Load libsgpeaks.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2210_14313_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.sgp_launch.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                 dp, dp]
        L.sgp_launch.restype = ctypes.c_int32
        L.sgp_op_name.argtypes = [ctypes.c_int32]
        L.sgp_op_name.restype = ctypes.c_char_p
        _lib = L
    return _lib


def measure(blocks: int = 0, iters: int = 4096, reps: int = 5, ops=None):
    """Per-class rates on cuda:0: {name: {"ops_per_s", "flops_per_s",
    "ms_per_launch", "ops_per_launch"}}.  blocks = 0 picks 8 workgroups of 4
    waves per compute unit (8 waves per SIMD)."""
    import torch
    L = lib()
    dev = torch.device("cuda:0")
    if blocks <= 0:
        blocks = 8 * torch.cuda.get_device_properties(dev).multi_processor_count
    sink = torch.zeros(blocks, dtype=torch.float64, device=dev)
    s = torch.cuda.Stream()
    res = {}
    for name in (ops or list(OPS)):
        op = OPS[name]
        n_ops, fpo = ctypes.c_double(), ctypes.c_double()

        def launch():
            rc = L.sgp_launch(op, blocks, iters, ctypes.c_void_p(sink.data_ptr()), ctypes.c_void_p(s.cuda_stream),
                              ctypes.byref(n_ops), ctypes.byref(fpo))
            if rc != 0:
                raise RuntimeError(f"sgp_launch({name}) failed with status {rc}")

        launch()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            launch()
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        rate = n_ops.value / (ms / 1e3)
        res[name] = {"ops_per_s": rate, "flops_per_s": rate * fpo.value, "ms_per_launch": ms,
                     "ops_per_launch": n_ops.value, "blocks": blocks, "iters": iters}
    return res
