"""Benchmark: batched Smolyak quadrature on one MI355X.

One step = one forward launch of the whole batched path over the
4096-integrand uneven workload (d ~ U{8..256}, K = q-d ~ U{2..6},
Clenshaw-Curtis / Gauss-Legendre, oscillatory / exp-sum), FP32-compensated
per-coordinate arithmetic with FP64 sweep products, a-priori error bound
computed for every result.  Inputs are resident in HBM before timing.

Prints ONE JSON line (rank 0).  Metric: effective sparse-grid points per
second = sum over integrands of n_d^q (points with repetition of (2.6))
divided by the time of one step.  Extras: time-to-integral at d = 1000,
batched vs plain per-integrand FP64 speedup at the 1e-7 accuracy target,
the FP64 batched rate, and the accuracy against the CPU oracle's values
of the timed workloads, stored under tests/golden (the oracle itself runs
only for the CPU baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published MI355X vector peaks (data sheet): FP32 157.3 TFLOP/s (with packed
# FP32 math), FP64 78.6 TFLOP/s; the transcendental unit taken at a quarter of
# the FP32 rate.  The roofline itself uses ceilings measured on the device by
# libsgpeaks.so (see measured_ceilings); these give a second, data-sheet
# fraction beside it.
PUBLISHED_PEAKS = {"fp32_flops_per_s": 157.3e12, "fp64_flops_per_s": 78.6e12,
                   "transcendentals_per_s": 157.3e12 / 4}
# non-packed VALU rate at the data-sheet clock: 256 CUs x 4 SIMDs x 16 lanes x
# 2 flops (FMA) x 2.4 GHz (the unit of the older flop-slot count below)
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PAIR_EVAL_FLOPS = 8.0   # flop-slot count: one centred node-pair evaluation = one quarter-rate slot


# HBM traffic of one forward launch on the 4096-integrand batch, from two
# rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE per dispatch) scaled by
# what the same counters read for a device copy of known size (bench.py
# --copy-probe-mb), keyed by precision and by a hash of the kernel sources
# the counters were taken on; any other source hash reports null.
MEASURED_TRAFFIC = {
    ("fp32c", "42138974188eff10"): 8257726.0,
}

# SQ_ACTIVE_INST_VALU of one forward launch on the same batch (quad-cycles
# summed over the SIMDs, median dispatch of a rocprofv3 --pmc pass), keyed
# like MEASURED_TRAFFIC.  With this run's launch time it gives the fraction
# of the launch's SIMD cycles that issue VALU work (4 cycles per
# quad-cycle, 4 SIMDs per compute unit, the 2.4 GHz engine clock).
MEASURED_VALU_ACTIVE = {
    ("fp32c", "42138974188eff10"): 2824990.0,
}


# The headline plan's schedule, pinned so that the headline and its
# rocprofv3 profile run the same launch shape: the balanced schedule with two
# waves per SIMD (the library's default; the autotuner's choice on this batch
# lands within a few per cent of it).  A tuple (coords_per_lane, max_group,
# cost_scaled, persistent, graph) names a coordinates-per-lane schedule.
PINNED_SCHEDULE = {"fp32c": ("balanced", 2, 0), "fp32e": ("balanced", 2, 0), "fp64": ("balanced", 2, 0)}


def kernel_source_hash() -> str:
    """Hash of the sources the headline forward kernel is built from: its
    device code and tables, and the forward descriptor layout (the part of
    sg_internal.hpp from FwdSeg to FwdWG)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2210_14313_amd", "csrc")
    for f in ("sg_device.hpp", "sg_fwd_inst.hpp", "sg_fwd_p1_k6.hip", "sg_rules.cpp", "gen_tables.cpp"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(csrc, "sg_internal.hpp"), "rb") as fh:
        text = fh.read()
    a = text.index(b"struct FwdSeg {")
    b = text.index(b"};", text.index(b"struct FwdWG {")) + 2
    h.update(text[a:b])
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def torch_device_cu_count() -> int:
    """Compute units of the current device."""
    import torch
    return int(torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count)


def copy_probe(mb: int) -> None:
    """Calibration workload for the traffic counters: five device-to-device
    copies of `mb` MiB (each reads and writes mb MiB)."""
    import torch
    n = mb * (1 << 20) // 8
    x = torch.empty(n, dtype=torch.float64, device="cuda:0").uniform_()
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 8, "copies": 5}))


def host_device_alias(host_ptr: int):
    """Device address of pinned host memory (hipHostGetDevicePointer), or
    None if the runtime does not map it."""
    import ctypes
    try:
        hip = ctypes.CDLL("libamdhip64.so")
    except OSError:
        return None
    d = ctypes.c_void_p()
    rc = hip.hipHostGetDevicePointer(ctypes.byref(d), ctypes.c_void_p(host_ptr), ctypes.c_uint(0))
    return d.value if rc == 0 and d.value else None


def algorithmic_flops(info) -> float:
    """Flop-slots of one forward launch: pair evaluations x 8 + 2 x MACs +
    sweep merge flops (see the plan info fields)."""
    return PAIR_EVAL_FLOPS * info["pair_evals"] + 2.0 * info["macs"] + info["merge_flops"]


def adjoint_flop_slots(info, problems) -> float:
    """Flop-slots of one reverse sweep: the forward surpluses and the
    derivative surpluses (each as in algorithmic_flops, without the merge),
    per unit the prefix, suffix and exclusion products of truncated
    polynomials (3 K^2) and the contraction with the derivative surpluses
    (2 K)."""
    surpl = PAIR_EVAL_FLOPS * info["pair_evals"] + 2.0 * info["macs"]
    per_unit = sum(p.d * (3 * (p.q - p.d) ** 2 + 2 * (p.q - p.d)) for p in problems)
    return 2.0 * surpl + float(per_unit)


def points_flop_slots(d: int, q: int, rule: str):
    """Points (with repetition) and algorithmic flop-slots of the literal
    point-by-point sum over the window of (2.6): per point one transcendental
    evaluation of f (8 slots, as for a node pair of the sweep), the
    multiply-add of w * (f(x) - f(c)) into the sum (2) and, over its nnz
    active coordinates, nnz - 1 additions forming the partial quantity and
    nnz multiplications forming coefficient times weight.  Exact integers
    from the per-level node counts by generating functions in z (excess):
    N(z) = sum_e n_{e+1} z^e, points = sum_window [z^e] N^d,
    sum of nnz over points = d sum_window [z^e] (N - n_1) N^(d-1)."""
    from paper_2210_14313_amd import native
    K = q - d
    n = [len(native.rule_table(rule, e + 1)[0]) for e in range(K + 1)]

    def mul(a, b):
        r = [0] * (K + 1)
        for i, x in enumerate(a):
            if x:
                for j in range(K + 1 - i):
                    r[i + j] += x * b[j]
        return r

    def power(a, k):
        r = [1] + [0] * K
        while k:
            if k & 1:
                r = mul(r, a)
            a = mul(a, a)
            k >>= 1
        return r

    Nd1 = power(n, d - 1)
    Nd = mul(Nd1, n)
    M = [0] + n[1:]
    MN = mul(M, Nd1)
    lo = max(0, K - d + 1)
    pts = sum(Nd[lo:K + 1])
    nnz = d * sum(MN[lo:K + 1])
    return pts, 10 * pts + 2 * nnz - pts


def _rule_facts(rule: str, K: int):
    """(distinct nodes of levels 1..K+1, sum over e = 1..K of the number of
    nodes carrying non-zero weight in the difference rule J^{e+1} - J^e),
    from the library's 1-D rule tables."""
    from paper_2210_14313_amd import native
    key = (rule, K)
    if key not in _RULE_FACTS:
        levels = [native.rule_table(rule, lv) for lv in range(1, K + 2)]
        union = {round(float(x), 14) for x, _ in levels for x in x}
        supp = 0
        for e in range(1, K + 1):
            wsum = {}
            for sign, (xs, ws) in ((1.0, levels[e]), (-1.0, levels[e - 1])):
                for x, w in zip(xs, ws):
                    k = round(float(x), 14)
                    wsum[k] = wsum.get(k, 0.0) + sign * float(w)
            supp += sum(1 for v in wsum.values() if v != 0.0)
        _RULE_FACTS[key] = (len(union), supp)
    return _RULE_FACTS[key]


_RULE_FACTS = {}


def method_counts(problems):
    """Operations the dimension sweep must execute for a batch, per
    (integrand, coordinate) unit summed over the batch, independent of how a
    kernel implements them: one transcendental per node of the union of the
    levels' node sets (two for the oscillatory family, whose factor e^{i a x}
    is complex), 2 FP32 flops per node carrying weight in a difference rule
    J^{e+1} - J^e, e = 1..K (times 2 when complex), and the FP64 flops of one
    truncated-polynomial product of K + 1 coefficients, (K + 1)(K + 2)
    (times 4 when complex)."""
    nt = n32 = n64 = 0
    for p in problems:
        K = p.q - p.d
        nodes, supp = _rule_facts(p.rule, K)
        cx = p.family in ("oscillatory", "oscillatory_quadratic", "oscillatory_quadratic_linear")
        nt += p.d * nodes * (2 if cx else 1)
        n32 += p.d * 2 * supp * (2 if cx else 1)
        n64 += p.d * (K + 1) * (K + 2) * (4 if cx else 1)
    return {"transcendentals": float(nt), "fp32_flops": float(n32), "fp64_flops": float(n64)}


def measured_ceilings():
    """Per-class VALU ceilings measured on this device (libsgpeaks.so): the
    best rate among the encodings of each class."""
    from paper_2210_14313_amd import peaks
    m = peaks.measure()
    return {"transcendentals_per_s": max(m[k]["ops_per_s"] for k in ("v_exp_f32", "v_sin_f32", "v_cos_f32")),
            "fp32_flops_per_s": max(m[k]["flops_per_s"] for k in ("v_fmac_f32", "v_fma_f32")),
            "fp64_flops_per_s": max(m[k]["flops_per_s"] for k in ("v_fmac_f64", "v_fma_f64")),
            "probe": {k: {"ops_per_s": v["ops_per_s"], "flops_per_s": v["flops_per_s"]} for k, v in m.items()}}


_CEILINGS = None


def ceilings():
    """measured_ceilings(), measured once per process."""
    global _CEILINGS
    if _CEILINGS is None:
        _CEILINGS = measured_ceilings()
    return _CEILINGS


def adjoint_counts(problems):
    """Operations of the reverse sweep: the forward work (node values and
    their difference-rule sums, one truncated product per unit), the same
    again for the derivative node values, and two more truncated products per
    unit (the exclusive prefix and suffix products whose product is the
    coefficient of a coordinate's surpluses)."""
    c = method_counts(problems)
    return {"transcendentals": 2 * c["transcendentals"], "fp32_flops": 2 * c["fp32_flops"],
            "fp64_flops": 3 * c["fp64_flops"]}


def serial_issue_roofline(counts, ceil, kernel_s):
    """Serial-issue model: T_min = sum over classes of count / ceiling;
    frac = T_min / kernel time.  achieved and peak are in FP32-equivalent
    TFLOP/s (T_min expressed at the FP32 ceiling), so achieved / peak = frac."""
    parts = {"transcendental": counts["transcendentals"] / ceil["transcendentals_per_s"],
             "fp32": counts["fp32_flops"] / ceil["fp32_flops_per_s"],
             "fp64": counts["fp64_flops"] / ceil["fp64_flops_per_s"]}
    tmin = sum(parts.values())
    peak = ceil["fp32_flops_per_s"] / 1e12
    frac = tmin / kernel_s
    return {"bound": "alu", "achieved": frac * peak, "peak": peak, "unit": "TFLOP/s", "frac": frac,
            "t_min_us": tmin * 1e6, "t_min_parts_us": {k: v * 1e6 for k, v in parts.items()},
            "kernel_us": kernel_s * 1e6}


BENCH_REFS = os.path.join(ROOT, "tests", "golden", "bench_refs.npz")


def bench_refs():
    """The oracle's values for the timed workloads, stored by
    tests/golden/make_bench_refs.py (the benchmark itself runs the oracle
    only for its CPU baseline)."""
    import numpy as np
    with np.load(BENCH_REFS) as z:
        return {k: z[k] for k in z.files}


def adjoint_leg(dev, s):
    """Reverse sweep on the 256-integrand oscillatory d = 200, q = 205 CC
    batch: gradient and forward time per launch (HIP events on the launch
    stream), error against the oracle's binary128 gradient of the first 64
    integrands (stored), roofline over the reverse sweep's flop-slots."""
    import numpy as np
    import torch

    from paper_2210_14313_amd import api, native, workloads as W
    gb = W.gradient_osc_d200()
    gref = bench_refs()["gradient_osc_d200_first64"]
    gparams = api.params_tensor(gb, dev)
    gout = torch.ones(len(gb), dtype=torch.float64, device=dev)
    adj = {}
    for prec in ("fp32c", "fp64"):
        plan = native.Plan(gb.problems, prec)
        gp = torch.zeros_like(gparams)
        s.wait_stream(torch.cuda.current_stream())
        for _ in range(3):
            plan.execute_grad(gparams, gout, gp, stream=s)
        torch.cuda.synchronize()
        reps = 50
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            plan.execute_grad(gparams, gout, gp, stream=s)
        e1.record(s)
        torch.cuda.synchronize()
        fwd = torch.empty(len(gb), dtype=torch.float64, device=dev)
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f0.record(s)
        for _ in range(reps):
            plan.execute(gparams, fwd, stream=s)
        f1.record(s)
        torch.cuda.synchronize()
        g = gp.cpu().numpy()
        errs = []
        for i, p in enumerate(gb.problems[:len(gref)]):
            sl = slice(p.param_offset, p.param_offset + p.d + 1)
            errs.append(np.max(np.abs(g[sl] - gref[i])) / np.max(np.abs(gref[i])))
        gms = e0.elapsed_time(e1) / reps
        slots = adjoint_flop_slots(plan.info(), gb.problems)
        roof = serial_issue_roofline(adjoint_counts(gb.problems), ceilings(), gms / 1e3)
        roof["frac_flop_slots"] = slots / (gms / 1e3) / 1e12 / VALU_PEAK_TFLOPS
        adj[prec] = {"grad_ms": gms, "forward_ms": f0.elapsed_time(f1) / reps,
                     "max_rel_err_vs_oracle_grad": float(np.max(errs)), "checked_integrands": len(errs),
                     "roofline": roof}
        plan.close()
    return adj


def oscq_leg(dev, s, reps: int = 50):
    """Oscillatory quadratic cos(2 pi w + sum a_i (x_i - u_i)^2) on the sweep
    with complex surpluses (sg_integrate, FP64, and the FP32 modes beside it),
    d = 1000, q = 1004,
    Gauss-Patterson: time per call (HIP events on the launch stream),
    accuracy against the oracle's stored binary128 value, and the roofline
    over its flop-slots (two sincos per node pair, 16; 4 per complex
    multiply-add of a surplus; 4 K^2 per coordinate for the complex
    truncated products).  One integrand is one workgroup: the launch is
    latency-bound by construction."""
    import torch
    from paper_2210_14313_amd import api, native, workloads as W
    b = W.oscillatory_quadratic_d1000()
    p = b.problems[0]
    K = p.q - p.d
    pr = api.params_tensor(b, dev)
    o = torch.empty(1, dtype=torch.float64, device=dev)
    bd = torch.empty_like(o)
    s.wait_stream(torch.cuda.current_stream())
    for _ in range(3):
        native.integrate_one(p, pr, "fp64", out=o, bound=bd, stream=s)
    torch.cuda.synchronize()
    # through the Python binding: the host's per-call cost sets the pace
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        native.integrate_one(p, pr, "fp64", out=o, bound=bd, stream=s)
    e1.record(s)
    torch.cuda.synchronize()
    ms_binding = e0.elapsed_time(e1) / reps
    # the C entry point with its arguments marshalled once: the launches
    # queue faster than they run, so the events time the kernel
    import ctypes
    lib, ctx = native.lib(), native.default_context()
    cp = native.SgProblem(p.d, p.q, native.RULES[p.rule], native.FAMILIES[p.family], 0)
    args = (ctx.handle, ctypes.byref(cp), native.PRECISIONS["fp64"], ctypes.c_void_p(pr.data_ptr()),
            ctypes.c_void_p(o.data_ptr()), ctypes.c_void_p(bd.data_ptr()), ctypes.c_void_p(s.cuda_stream))
    torch.cuda.synchronize()
    e0.record(s)
    bad = sum(1 for _ in range(reps) if lib.sg_integrate(*args) != 0)
    e1.record(s)
    torch.cuda.synchronize()
    assert bad == 0, "sg_integrate failed"
    ms = e0.elapsed_time(e1) / reps
    refs = bench_refs()
    ref = float(refs["oscq_d1000"][0])
    # the same rule tables as a real family of the same shape: its plan's counts
    plan = native.Plan([W.Problem(p.d, p.q, p.rule, "oscillatory", 0)], "fp64")
    info = plan.info()
    plan.close()
    slots = 2 * PAIR_EVAL_FLOPS * info["pair_evals"] + 4.0 * info["macs"] + 4.0 * K * K * p.d
    roof = serial_issue_roofline(method_counts(b.problems), ceilings(), ms / 1e3)
    roof["frac_flop_slots"] = slots / (ms / 1e3) / 1e12 / VALU_PEAK_TFLOPS
    sc = float(refs["oscq_d1000_scale"][0])      # modulus of the complex Smolyak sum
    res = {"d": p.d, "q": p.q, "rule": p.rule, "us_per_call": ms * 1e3, "us_per_call_python_binding": ms_binding * 1e3,
           "points_per_s": float(info["effective_points"]) / (ms / 1e3),
           "value": o.item(), "rel_err_vs_oracle": abs(o.item() - ref) / sc, "stated_bound_rel": bd.item() / sc,
           "roofline": roof}
    # the FP32 modes (FP32 node values, FP64 complex products), same entry point
    for prec in ("fp32c", "fp32e"):
        args = (ctx.handle, ctypes.byref(cp), native.PRECISIONS[prec], ctypes.c_void_p(pr.data_ptr()),
                ctypes.c_void_p(o.data_ptr()), ctypes.c_void_p(bd.data_ptr()), ctypes.c_void_p(s.cuda_stream))
        for _ in range(3):
            lib.sg_integrate(*args)
        torch.cuda.synchronize()
        e0.record(s)
        bad = sum(1 for _ in range(reps) if lib.sg_integrate(*args) != 0)
        e1.record(s)
        torch.cuda.synchronize()
        assert bad == 0, "sg_integrate failed"
        m2 = e0.elapsed_time(e1) / reps
        res[prec] = {"us_per_call": m2 * 1e3, "value": o.item(), "rel_err_vs_oracle": abs(o.item() - ref) / sc,
                     "stated_bound_rel": bd.item() / sc}
    log(f"  oscillatory quadratic d={p.d}: {ms * 1e3:.2f} us per call, err {res['rel_err_vs_oracle']:.2e}; "
        f"fp32c {res['fp32c']['us_per_call']:.2f} us, err {res['fp32c']['rel_err_vs_oracle']:.2e}")
    return res


def points_leg(dev, s, reps: int = 5):
    """Time the literal point-by-point path on the d = 100, q = 105
    Clenshaw-Curtis workload (both families) and check it against the
    stored full-size oracle values; roofline in flop-slots per launch."""
    import torch
    from paper_2210_14313_amd import api, native, workloads as W
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_full_size.json")))["rows"]
    pd100 = W.precision_d100()
    pts = {}
    for row in [r for r in golden if r["workload"] == "precision_d100"]:
        one = pd100.subset([row["index"]])
        p = one.problems[0]
        pr = api.params_tensor(one, dev)
        o = torch.empty(1, dtype=torch.float64, device=dev)
        bd = torch.empty(1, dtype=torch.float64, device=dev)
        native.integrate_points(p, pr, out=o, bound=bd, stream=s)     # warm
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            native.integrate_points(p, pr, out=o, bound=bd, stream=s)
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        npts, slots = points_flop_slots(p.d, p.q, p.rule)
        assert npts == int(row["npoints"]), (npts, row["npoints"])
        ref_pt = row["points_hi"] + row["points_lo"]
        sc = float(bench_refs()["precision_d100_scale"][row["index"]])   # oracle accuracy scale
        # per point one transcendental evaluation of f and, in FP64, the
        # multiply-add into the sum plus, over its active coordinates, the
        # additions of the partial quantity and the weight products
        nnz = (slots - 9 * npts) // 2
        roof = serial_issue_roofline({"transcendentals": float(npts), "fp32_flops": 0.0,
                                      "fp64_flops": float(npts + 2 * nnz)}, ceilings(), ms / 1e3)
        roof["frac_flop_slots"] = slots / (ms / 1e3) / 1e12 / VALU_PEAK_TFLOPS
        pts[p.family] = {"points": float(npts), "ms": ms, "points_per_s": npts / (ms / 1e3),
                         "rel_err_vs_point_oracle": abs(o.item() - ref_pt) / sc,
                         "stated_bound_rel": bd.item() / sc, "roofline": roof}
        log(f"  points {p.family}: {ms:.2f} ms, {npts / (ms / 1e3):.3e} points/s, frac {roof['frac']:.4f}")
    return pts


def blocked_leg(dev, s, batch, precision: str, m: int = 10, reps: int = 50):
    """Block (tensor-product) variant of the rule, Algorithm 3.3 with step m:
    the batch in blocks of m coordinates (block gather, forward over the
    blocks, ordered combine; timed with events, roofline over the forward
    work of the blocks, accuracy against the oracle's block rule on the
    first 256 integrands of the 4096 batch, stored), and the m = 10 setting
    of Table 4.9
    (Gauss-Legendre with n_l = l, [-1,1]^d mapped to the unit cube; excess
    K = 8, the largest this library builds, where the table uses 9): time
    to integral and relative error against the exact integral."""
    import numpy as np
    import torch
    from paper_2210_14313_amd import api, native, workloads as W
    refs = bench_refs()
    res = {}
    params = api.params_tensor(batch, dev)
    plan = native.Plan(batch.problems, precision, block_dims=m)
    out = torch.empty(len(batch), dtype=torch.float64, device=dev)
    bound = torch.empty_like(out)
    plan.autotune(params, out, stream=s)      # the blocks form a different batch shape
    for _ in range(5):
        plan.execute(params, out, bound, stream=s)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        plan.execute(params, out, bound, stream=s)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    info = plan.info()
    plan.close()
    got, bnd = out.cpu().numpy(), bound.cpu().numpy()
    if len(batch) == 4096 and m == 10:
        ref = refs["blocked_m10_first256"]
        idx = list(range(len(ref)))
        sc = refs["blocked_m10_first256_scale"]      # oscillatory: modulus of the complex block rule
        acc_err = float(np.max(np.abs(got[idx] - ref) / sc))
        acc_ok = bool(np.all(np.abs(got[idx] - ref) <= bnd[idx]))
    else:
        idx, acc_err, acc_ok = [], None, None
    roof = serial_issue_roofline(method_counts(batch.problems), ceilings(), ms / 1e3)
    roof["frac_flop_slots"] = algorithmic_flops(info) / (ms / 1e3) / 1e12 / VALU_PEAK_TFLOPS
    res[f"batched_uneven_{len(batch)}_m{m}"] = {
        "precision": precision, "ms_per_launch": ms, "block_subproblems_units": info["units"],
        "schedule": {k: info[k] for k in ("coords_per_lane", "max_group", "cost_scaled", "persistent", "graph",
                                          "grid_blocks", "balanced")},
        "roofline": roof,
        "max_rel_err_vs_block_oracle": acc_err, "all_within_stated_bound": acc_ok,
        "checked_integrands": len(idx)}
    log(f"  blocked m={m} {precision}: {ms * 1e3:.2f} us per launch, frac {roof['frac']:.4f}")
    K = 8
    paper = {}
    # exp(sum (-1)^(i+1) x_i) at d = 1000; prod 1/(0.9^2 + (x_i - 0.6)^2) at
    # d = 300 (on the unit cube its value exceeds the double range at d = 1000)
    names = [str(x) for x in refs["table_4_9_names"]]
    for name, fam, d in (("exp_alt_d1000", "exp_sum", 1000), ("peak_06_d300", "product_peak", 300)):
        prm = (np.array([2.0 * (-1) ** i for i in range(d)]) if fam == "exp_sum"
               else np.concatenate([np.full(d, 1 / 0.45), np.full(d, 0.8)]))
        one = W.single(d, d + K, "gl_paper", fam, prm)
        pr = api.params_tensor(one, dev)
        row = {}
        for prec in ("fp64", "fp32c"):
            plan = native.Plan(one.problems, prec, block_dims=10)
            o = torch.empty(1, dtype=torch.float64, device=dev)
            bo = torch.empty(1, dtype=torch.float64, device=dev)
            ts = []
            with torch.cuda.stream(s):
                for k in range(31):
                    t0 = time.perf_counter()
                    plan.execute(pr, o, bo, stream=s)
                    v = o.item()
                    ts.append(time.perf_counter() - t0)
            plan.close()
            ex = float(refs["table_4_9_exact"][names.index(name)])
            orc_v = float(refs["table_4_9_blocked"][names.index(name)])
            row[prec] = {"value": v, "stated_bound": bo.item(), "time_to_integral_median_s": statistics.median(ts[1:]),
                         "rel_err_vs_exact": abs((v - ex) / ex),
                         "rel_diff_vs_block_oracle": abs(v - orc_v) / abs(orc_v)}
        paper[name] = row
        log(f"  blocked m=10 {name}: rel err vs exact {row['fp64']['rel_err_vs_exact']:.4e}, "
            f"{row['fp64']['time_to_integral_median_s'] * 1e6:.1f} us")
    res["table_4_9_setting_m10_gl_K8"] = paper
    return res


def plain_leg(dev, s, batch, params, main_run, accuracy):
    """The plain per-integrand FP64 path (sg_integrate: one launch per
    integrand, no plan, no graph) over the whole batch, against one launch of
    the batched plan.  Three times for the plain path: wall time through the
    Python binding, wall time calling the C entry point with its arguments
    marshalled beforehand, and the device time (HIP events on the launch
    stream around every launch, summed).  The speedup is reported only when
    the batched result meets the 1e-7 target against the oracle's accuracy
    scale in the same run."""
    import ctypes
    import numpy as np
    import torch
    from paper_2210_14313_amd import native, workloads as W
    log("plain per-integrand FP64 path ...")
    outp = torch.empty(len(batch), dtype=torch.float64, device=dev)
    s.wait_stream(torch.cuda.current_stream())
    views = [(p, params[p.param_offset: p.param_offset + W.n_params(p.family, p.d)], outp[i: i + 1])
             for i, p in enumerate(batch.problems)]
    for p, pv, ov in views[:64]:
        native.integrate_one(p, pv, "fp64", out=ov, stream=s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, pv, ov in views:
        native.integrate_one(p, pv, "fp64", out=ov, stream=s)
    torch.cuda.synchronize()
    t_binding = time.perf_counter() - t0
    # the C entry point, arguments marshalled once
    lib, ctx = native.lib(), native.default_context()
    cps = [native.SgProblem(p.d, p.q, native.RULES[p.rule], native.FAMILIES[p.family], 0) for p, _, _ in views]
    args = [(ctx.handle, ctypes.byref(cp), native.PRECISIONS["fp64"], ctypes.c_void_p(pv.data_ptr()),
             ctypes.c_void_p(ov.data_ptr()), None, ctypes.c_void_p(s.cuda_stream))
            for cp, (_, pv, ov) in zip(cps, views)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bad = sum(1 for a in args if lib.sg_integrate(*a) != 0)
    torch.cuda.synchronize()
    t_c = time.perf_counter() - t0
    assert bad == 0, "sg_integrate failed"
    # device time: an event pair around every launch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in args]
    torch.cuda.synchronize()
    for (e0, e1), a in zip(ev, args):
        e0.record(s)
        lib.sg_integrate(*a)
        e1.record(s)
    torch.cuda.synchronize()
    t_dev = sum(e0.elapsed_time(e1) for e0, e1 in ev) / 1e3
    got = outp.cpu().numpy()
    acc_b = accuracy(main_run["got"], main_run["bound"])
    acc_p = accuracy(got, np.full_like(got, np.inf))
    ok = acc_b is not None and acc_b["max_rel_err_vs_oracle"] <= 1e-7
    bms = main_run["ms_per_step"]
    return {"plain_fp64_ms_binding": t_binding * 1e3, "plain_fp64_ms_c_abi": t_c * 1e3,
            "plain_fp64_ms_device": t_dev * 1e3, "batched_ms": bms, "batched_kernel_ms": main_run["kernel_ms"],
            "speedup": (t_binding * 1e3 / bms) if ok else None,
            "speedup_c_abi": (t_c * 1e3 / bms) if ok else None,
            "speedup_device": (t_dev * 1e3 / main_run["kernel_ms"]) if ok else None,
            "batched_max_rel_err": None if acc_b is None else acc_b["max_rel_err_vs_oracle"],
            "plain_max_rel_err": None if acc_p is None else acc_p["max_rel_err_vs_oracle"],
            "plain_per_family": None if acc_p is None else
            {f: {k: v[k] for k in ("max_rel_err_vs_oracle", "max_plain_rel_err")} for f, v in acc_p["per_family"].items()},
            "accuracy_target": 1e-7, "accuracy_scale": "oracle accuracy scale (oscillatory: complex modulus)"}


def host_cpu():
    """nproc, the CPUs this process may run on, and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model}


def host_threads() -> int:
    """Oracle threads for the CPU baseline: every CPU this process may run
    on, at most 16 (the host share of one GPU on the measurement machines)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def cpu_baseline(batch, target_points: float, threads: int):
    """Time the point-by-point oracle on the first integrands of the batch
    (skipping any with more than 5e8 points) until ~target_points are done."""
    import oracle
    from oracle import counts as OC
    idx, total = [], 0
    for i, p in enumerate(batch.problems):
        n = OC.counts_by_generating_function(p.d, p.q, p.rule)["n_points_rep"]
        if n > 5e8:
            continue
        idx.append((i, n))
        total += n
        if total >= target_points:
            break
    t0 = time.perf_counter()
    done = 0
    for i, n in idx:
        p = batch.problems[i]
        r = oracle.smolyak_points(p.d, p.q, p.rule, p.family, batch.param_slice(i), nthreads=threads)
        done += r["npoints"]
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "points/s", "cores": threads, "kind": "oracle", "host": host_cpu(),
            "sample": f"first {len(idx)} integrands of the batch with n_d^q <= 5e8 "
                      f"({done:.3e} points, {dt:.1f} s, point-by-point (2.6)-(2.7) in x87 extended precision)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp32c", choices=["fp32c", "fp32e", "fp64"])
    ap.add_argument("--n", type=int, default=4096, help="integrands in the batch")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the headline plan instead of using the pinned schedule")
    ap.add_argument("--no-autotune", action="store_true", help="extras: use default schedules, no autotuning")
    ap.add_argument("--sched", default="",
                    help="headline plan's schedule: coords_per_lane,max_group,cost_scaled,persistent,graph "
                         "(default: the autotuner's usual choice for the 4096 batch, pinned)")
    ap.add_argument("--balanced", type=int, default=0,
                    help="headline plan's schedule: the balanced schedule with this many waves per SIMD")
    ap.add_argument("--cpu-points", type=float, default=1.5e9)
    ap.add_argument("--scaling-mults", default="16,64",
                    help="extra batch sizes (multiples of --n) for the scaling series")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="only run the traffic-counter calibration copy of this many MiB")
    ap.add_argument("--blocked-only", action="store_true",
                    help="only run the block-variant leg (m = 10) and print its JSON")
    ap.add_argument("--oscq-only", action="store_true",
                    help="only the oscillatory-quadratic sweep leg (d = 1000)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the reverse-sweep leg (oscillatory d = 200, 256 integrands)")
    ap.add_argument("--points-only", action="store_true",
                    help="only run the literal point-by-point leg (d = 100, q = 105) and print its JSON")
    args = ap.parse_args()
    if args.copy_probe_mb > 0:
        copy_probe(args.copy_probe_mb)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(a batch of independent integrands would be split across GPUs by cost, "
              "with no communication); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2210_14313_amd import api, native, workloads as W

    if args.oscq_only:
        torch.cuda.set_device(0)
        so = torch.cuda.Stream()
        print(json.dumps({"oscillatory_quadratic_d1000": oscq_leg(torch.device("cuda:0"), so)}), flush=True)
        return

    if args.adjoint_only:
        torch.cuda.set_device(0)
        sa = torch.cuda.Stream()
        print(json.dumps({"adjoint_gradient_osc_d200_n256": adjoint_leg(torch.device("cuda:0"), sa)}), flush=True)
        return

    if args.points_only:
        torch.cuda.set_device(0)
        sp = torch.cuda.Stream()
        print(json.dumps({"points_path_precision_d100": points_leg(torch.device("cuda:0"), sp)}), flush=True)
        return

    batch = W.batched_uneven(n=args.n)
    if args.blocked_only:
        torch.cuda.set_device(0)
        sb = torch.cuda.Stream()
        print(json.dumps({"blocked_m10": blocked_leg(torch.device("cuda:0"), sb, batch, args.precision)}), flush=True)
        return
    # accuracy statement against the oracle's binary128 values of the
    # 4096-integrand batch (stored; other sizes report none)
    # errors are stated against the oracle's accuracy scale: |Q|, and for the
    # oscillatory family the modulus sqrt(Q(w)^2 + Q(w - 1/4)^2) of the
    # complex Smolyak sum (stored with the values); the plain |err| / |Q| is
    # reported beside it
    refs = bench_refs() if args.n == 4096 else None
    ref = refs["uneven_4096"] if refs else None
    scale = refs["uneven_4096_scale"] if refs else None
    fam = np.array([p.family for p in batch.problems])

    def rel_err(got):
        return None if ref is None else float(np.max(np.abs(got - ref) / scale))

    def within(got, bnd):
        return None if ref is None else bool(np.all(np.abs(got - ref) <= bnd))

    def accuracy(got, bnd):
        if ref is None:
            return None
        err = np.abs(got - ref)
        res = {"max_rel_err_vs_oracle": float(np.max(err / scale)), "all_within_stated_bound": within(got, bnd),
               "max_stated_rel_bound": float(np.max(bnd / scale)), "scale": "oracle accuracy scale",
               "per_family": {}}
        for f in sorted(set(fam)):
            sel = fam == f
            res["per_family"][f] = {
                "max_rel_err_vs_oracle": float(np.max(err[sel] / scale[sel])),
                "max_plain_rel_err": float(np.max(err[sel] / np.abs(ref[sel]))),
                "max_stated_rel_bound": float(np.max(bnd[sel] / scale[sel])),
                "max_bound_over_err": float(np.max(bnd[sel]) / max(float(np.max(err[sel])), 1e-300)),
                # per integrand (those with a non-zero error): how far each
                # stated bound is above its own error
                "median_bound_over_err": float(np.median(bnd[sel][err[sel] > 0] / err[sel][err[sel] > 0]))
                if np.any(err[sel] > 0) else None,
                "integrands": int(np.sum(sel))}
        return res

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    params = api.params_tensor(batch, dev)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()

    def run_plan(precision, steps, warmup, autotune, sched=None):
        plan = native.Plan(batch.problems, precision)
        out = torch.empty(len(batch), dtype=torch.float64, device=dev)
        bound = torch.empty_like(out)
        if sched and sched[0] == "balanced":
            plan.set_balanced(sched[1], graph=bool(sched[2]))
        elif sched:
            c, g, cs, pq, gr = sched
            plan.set_schedule(c, g, graph=bool(gr), persistent=bool(pq), cost_scaled=bool(cs))
        elif autotune:
            plan.autotune(params, out, stream=s)
        for _ in range(warmup):
            plan.execute(params, out, bound, stream=s)
        torch.cuda.synchronize()
        # Timed region: `steps` back-to-back launches on stream s, bracketed by
        # a device synchronisation on both sides; two HIP events on s around
        # the launches give the device time, and the average launch duration
        # is that time over the number of launches (the kernel is the only
        # work on s, so the figure includes no host time once the host keeps
        # ahead of the device).
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(s)
        for k in range(steps):
            plan.execute(params, out, bound, stream=s)
        e1.record(s)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kern_ms = e0.elapsed_time(e1) / steps
        got = out.cpu().numpy()
        bnd = bound.cpu().numpy()
        info = plan.info()
        log(f"  {precision}: sched cpl {info['coords_per_lane']} gmax {info['max_group']} cost_scaled "
            f"{info['cost_scaled']} persistent {info['persistent']} graph {info['graph']} balanced {info['balanced']} "
            f"grid {info['grid_blocks']}, kernel {kern_ms * 1e3:.2f} us, step {(t1 - t0) * 1e6 / steps:.2f} us")
        plan.close()
        return dict(ms_per_step=(t1 - t0) * 1e3 / steps, kernel_ms=float(kern_ms), got=got, bound=bnd, info=info)

    log(f"timing {args.precision} batched plan: {args.steps} steps after {args.warmup} warmup")
    if args.balanced:
        pinned = ("balanced", args.balanced, 0)
    elif args.sched:
        pinned = tuple(int(v) for v in args.sched.split(","))
    elif args.autotune:
        pinned = None
    else:
        pinned = PINNED_SCHEDULE[args.precision]
    main_run = run_plan(args.precision, args.steps, args.warmup, args.autotune, pinned)
    info = main_run["info"]
    max_err = rel_err(main_run["got"])
    eff = float(info["effective_points"])
    value = eff / (main_run["ms_per_step"] / 1e3)
    flops = algorithmic_flops(info)
    counts = method_counts(batch.problems)
    log("measuring per-operation VALU ceilings ...")
    ceil = ceilings()
    roof = serial_issue_roofline(counts, ceil, main_run["kernel_ms"] / 1e3)
    roof_pub = serial_issue_roofline(counts, PUBLISHED_PEAKS, main_run["kernel_ms"] / 1e3)
    valu_active = MEASURED_VALU_ACTIVE.get((args.precision, kernel_source_hash())) if args.n == 4096 else None
    n_simd = 4 * torch_device_cu_count()
    roof.update({
        "traffic": MEASURED_TRAFFIC.get((args.precision, kernel_source_hash())) if args.n == 4096 else None,
        "valu_busy_frac": (valu_active * 4.0 / n_simd / (main_run["kernel_ms"] * 1e-3 * 2.4e9)
                           if valu_active is not None else None),
        "model": "serial issue over operation classes, ceilings measured on this device",
        "counts": counts,
        "ceilings": {k: v for k, v in ceil.items() if k != "probe"},
        "ceiling_probe": ceil["probe"],
        "frac_published_peaks": roof_pub["frac"],
        "frac_flop_slots": flops / (main_run["kernel_ms"] / 1e3) / 1e12 / VALU_PEAK_TFLOPS,
        "flop_slots_per_launch": flops})
    log(f"  roofline frac {roof['frac']:.3f} (T_min {roof['t_min_us']:.2f} us), published peaks "
        f"{roof_pub['frac']:.3f}")
    result = {
        "metric": "sparse-grid points/s effective + time-to-integral d=1000; batched vs plain @1e-7",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32c": "f32c+f64", "fp32e": "f32+f64", "fp64": "f64"}[args.precision],
        "data": "synthetic (seeded integrand parameters, no dataset)",
        "config": {"workload": f"batched_uneven_{args.n}: d~U{{8..256}}, q-d~U{{2..6}}, rule~{{CC,GL(2l-1)}}, "
                               f"family~{{oscillatory, exp-sum}}, one launch per step",
                   "integrands": args.n, "precision": args.precision,
                   "schedule": {k: info[k] for k in ("coords_per_lane", "max_group", "cost_scaled", "persistent",
                                                     "graph", "grid_blocks", "balanced")},
                   "schedule_source": "pinned" if pinned else "autotuned",
                   "effective_points_per_step": eff, "parallelism": "single-gpu"},
        "roofline": roof,
        "accuracy": accuracy(main_run["got"], main_run["bound"]),
    }

    if not args.no_extras:
        extras = {}
        # the autotuner on the headline batch
        at = run_plan(args.precision, args.steps, 5, True)
        extras["autotuned_" + args.precision] = {
            "schedule": {k: at["info"][k] for k in ("coords_per_lane", "max_group", "cost_scaled", "persistent", "graph",
                                          "grid_blocks", "balanced")},
            "kernel_ms": at["kernel_ms"], "ms_per_step": at["ms_per_step"],
            "max_rel_err_vs_oracle": rel_err(at["got"])}
        # the same batch in the other launch forms: the balanced schedule
        # replayed from a captured graph, the coordinates-per-lane schedule
        # the work queue runs (direct), and the persistent work-queue kernel
        # (direct and in a graph), beside the headline's direct launch
        forms = {"balanced_direct": PINNED_SCHEDULE[args.precision]}
        forms["balanced_graph"] = ("balanced", 2, 1)
        forms["coords_per_lane_direct"] = (4, 4, 0, 0, 0)
        forms["persistent_queue_direct"] = (4, 4, 0, 1, 0)
        forms["persistent_queue_graph"] = (4, 4, 0, 1, 1)
        lf = {}
        for name, sched in forms.items():
            r2 = run_plan(args.precision, max(20, args.steps // 2), 5, False, sched)
            lf[name] = {"schedule": {k: r2["info"][k] for k in ("coords_per_lane", "max_group", "persistent", "graph",
                                                               "grid_blocks", "balanced")},
                        "kernel_ms": r2["kernel_ms"], "ms_per_step": r2["ms_per_step"],
                        "max_rel_err_vs_oracle": rel_err(r2["got"])}
        extras["launch_forms_" + args.precision] = lf
        # the other precision modes' batched rates
        for other in [m for m in ("fp64", "fp32e", "fp32c") if m != args.precision]:
            r2 = run_plan(other, max(20, args.steps // 2), 5, False, PINNED_SCHEDULE[other])
            extras[f"{other}_batched"] = {
                "points_per_s": eff / (r2["ms_per_step"] / 1e3), "ms_per_step": r2["ms_per_step"],
                "kernel_ms": r2["kernel_ms"], "max_rel_err_vs_oracle": rel_err(r2["got"]),
                "all_within_stated_bound": within(r2["got"], r2["bound"])}
        # plain per-integrand FP64 path: one launch per integrand, no plan, no graph
        extras["batched_vs_plain"] = plain_leg(dev, s, batch, params, main_run, accuracy)
        # time to integral at d = 1000 (wall time, call -> host-visible value)
        hd = W.high_dim_d1000()
        golden = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_full_size.json")))["rows"]
        ref_hd = {r["index"]: r["factorised_hi"] + r["factorised_lo"] for r in golden
                  if r["workload"] == "high_dim_d1000"}
        tti = {}
        for i, p in enumerate(hd.problems):
            one = hd.subset([i])
            pr = api.params_tensor(one, dev)
            for prec in ("fp32c", "fp64"):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                plan = native.Plan(one.problems, prec)
                o = torch.empty(1, dtype=torch.float64, device=dev)
                s.wait_stream(torch.cuda.current_stream())
                with torch.cuda.stream(s):
                    plan.execute(pr, o, stream=s)
                    v = o.item()              # copy on s, then host sync
                    cold = time.perf_counter() - t0
                    ts = []
                    for _ in range(30):
                        t0 = time.perf_counter()
                        plan.execute(pr, o, stream=s)
                        v = o.item()
                        ts.append(time.perf_counter() - t0)
                # result written by the kernel straight into pinned host memory
                # (its device alias from hipHostGetDevicePointer): call, then the
                # host polls the value (NaN until written; bounded wait, stream
                # synchronisation after each call either way)
                pinned = None
                hp = torch.empty(1, dtype=torch.float64, pin_memory=True)
                hv = hp.numpy()
                dptr = host_device_alias(hp.data_ptr())
                if dptr is not None:
                    tp = []
                    for _ in range(31):
                        hv[0] = float("nan")
                        t0 = time.perf_counter()
                        plan.execute_raw(pr.data_ptr(), dptr, None, stream=s)
                        while hv[0] != hv[0] and time.perf_counter() - t0 < 0.1:
                            pass
                        vp = float(hv[0])
                        tp.append(time.perf_counter() - t0)
                        s.synchronize()
                    pinned = {"median_s": statistics.median(tp[1:]), "value": vp}
                # device time of the plan's launch (events around 50 launches)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(s)
                for _ in range(50):
                    plan.execute(pr, o, stream=s)
                e1.record(s)
                torch.cuda.synchronize()
                plan_kernel_us = e0.elapsed_time(e1) / 50 * 1e3
                plan.close()
                # the plan-free entry point (sg_integrate: the integrand split
                # over ceil(d / 256) workgroups joined in a fixed order)
                import ctypes
                lib, ctx = native.lib(), native.default_context()
                cp = native.SgProblem(p.d, p.q, native.RULES[p.rule], native.FAMILIES[p.family], 0)
                with torch.cuda.stream(s):
                    to = []
                    for _ in range(31):
                        t0 = time.perf_counter()
                        native.integrate_one(p, pr, prec, out=o, stream=s)
                        vo = o.item()
                        to.append(time.perf_counter() - t0)
                e0.record(s)
                for _ in range(50):
                    lib.sg_integrate(ctx.handle, ctypes.byref(cp), native.PRECISIONS[prec], ctypes.c_void_p(pr.data_ptr()),
                                     ctypes.c_void_p(o.data_ptr()), None, ctypes.c_void_p(s.cuda_stream))
                e1.record(s)
                torch.cuda.synchronize()
                pf = {"median_s": statistics.median(to[1:]), "kernel_us": e0.elapsed_time(e1) / 50 * 1e3,
                      "value": vo, "pinned_result": None}
                if dptr is not None:
                    tp = []
                    for _ in range(31):
                        hv[0] = float("nan")
                        t0 = time.perf_counter()
                        lib.sg_integrate(ctx.handle, ctypes.byref(cp), native.PRECISIONS[prec],
                                         ctypes.c_void_p(pr.data_ptr()), ctypes.c_void_p(dptr), None,
                                         ctypes.c_void_p(s.cuda_stream))
                        while hv[0] != hv[0] and time.perf_counter() - t0 < 0.1:
                            pass
                        vp1 = float(hv[0])
                        tp.append(time.perf_counter() - t0)
                        s.synchronize()
                    pf["pinned_result"] = {"median_s": statistics.median(tp[1:]), "value": vp1}
                ex = float(ref_hd[i])
                pf["rel_err_vs_oracle"] = abs(vo - ex) / abs(ex)
                tti[f"{p.rule}_{prec}"] = {"median_s": statistics.median(ts), "cold_s": cold, "value": v,
                                           "rel_err_vs_oracle": abs(v - ex) / abs(ex), "pinned_result": pinned,
                                           "kernel_us": plan_kernel_us, "plan_free": pf}
        extras["time_to_integral_d1000"] = tti
        # block (tensor-product) variant, Algorithm 3.3 with step m = 10
        log("block variant (m = 10) ...")
        extras["blocked_m10"] = blocked_leg(dev, s, batch, args.precision)
        # reverse sweep on the gradient workload (256 oscillatory, d = 200, q = 205)
        extras["adjoint_gradient_osc_d200_n256"] = adjoint_leg(dev, s)
        # oscillatory quadratic on the complex sweep (one integrand, d = 1000)
        extras["oscillatory_quadratic_d1000"] = oscq_leg(dev, s)

        # literal point-by-point path on the d = 100, q = 105 workload
        # (2.08e10 points per integrand) against the stored oracle values
        log("point-by-point path ...")
        extras["points_path_precision_d100"] = points_leg(dev, s)

        # scaling series: the same recipe with more integrands per launch
        scal = {str(args.n): {"kernel_ms": main_run["kernel_ms"], "grid_blocks": info["grid_blocks"],
                              "points_per_s_kernel": eff / (main_run["kernel_ms"] / 1e3),
                              "roofline_frac": roof["frac"], "roofline_frac_flop_slots": roof["frac_flop_slots"]}}
        for mult in [int(m) for m in args.scaling_mults.split(",") if m]:
            nb = W.batched_uneven(n=args.n * mult)
            log(f"scaling series: {len(nb)} integrands ...")
            bp = api.params_tensor(nb, dev)
            plan = native.Plan(nb.problems, args.precision)
            o = torch.empty(len(nb), dtype=torch.float64, device=dev)
            bd = torch.empty_like(o)
            plan.autotune(bp, o, stream=s)
            for _ in range(3):
                plan.execute(bp, o, bd, stream=s)
            torch.cuda.synchronize()
            reps = 20
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(reps):
                plan.execute(bp, o, bd, stream=s)
            e1.record(s)
            torch.cuda.synchronize()
            kms = e0.elapsed_time(e1) / reps
            ni = plan.info()
            fl = algorithmic_flops(ni)
            scal[str(len(nb))] = {"kernel_ms": kms, "grid_blocks": ni["grid_blocks"],
                                  "coords_per_lane": ni["coords_per_lane"],
                                  "points_per_s_kernel": float(ni["effective_points"]) / (kms / 1e3),
                                  "roofline_frac": serial_issue_roofline(method_counts(nb.problems), ceil,
                                                                         kms / 1e3)["frac"],
                                  "roofline_frac_flop_slots": fl / (kms / 1e3) / 1e12 / VALU_PEAK_TFLOPS}
            plan.close()
            del bp, o, bd
        extras["scaling_" + args.precision] = scal
        result["extras"] = extras

    if not args.no_cpu_baseline:
        log("CPU baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(batch, args.cpu_points, host_threads())
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
