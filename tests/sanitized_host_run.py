"""Driver for the CPU sanitizer tests (test_sanitizers.py), run as a child
process with the AddressSanitizer runtime preloaded.

Loads the host-only build of the runtime (the C ABI with a host stand-in for
the HIP runtime and launchers that launch nothing) and drives every entry
point through its host logic: counts, rule tables, coefficients, unranking,
plan building and packing for mixed batches in every precision mode and
schedule, the block variant, graph bookkeeping, autotune, the plan-free
entry points and the argument checks.  With --oracle it also runs the
sanitized oracle.  Prints one JSON object (the host functions' results, for
comparison with the product library, and the statuses seen); any sanitizer
report aborts the process with a non-zero status.

Usage: sanitized_host_run.py HOSTSAN_LIB [--oracle | --fail-malloc | --tuning DIR]
(--fail-malloc: a context, plan and call sequence repeated with the n-th
allocation failing, n = 1, 2, ...)
"""
from __future__ import annotations

import ctypes
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

vp, i32, u64, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64


class Problem(ctypes.Structure):
    _fields_ = [("d", i32), ("q", i32), ("rule", i32), ("family", i32), ("param_offset", i64)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("effective_points", u64), ("units", u64), ("pair_evals", u64), ("macs", u64),
                ("merge_flops", u64), ("block_threads", i32), ("grid_blocks", i32),
                ("coords_per_lane", i32), ("max_group", i32), ("graph", i32), ("persistent", i32),
                ("cost_scaled", i32), ("balanced", i32), ("fp64_complex", i32), ("reserved", i32)]


NPARAMS = {0: lambda d: d, 1: lambda d: d + 1, 2: lambda d: 2 * d, 3: lambda d: d, 4: lambda d: 2 * d,
           5: lambda d: 2 * d + 1, 6: lambda d: 3 * d + 1}


def load(path):
    L = ctypes.CDLL(path)
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
        "sg_plan_create": ([vp, P(Problem), i32, i32, P(vp)], i32),
        "sg_plan_create_blocked": ([vp, P(Problem), i32, i32, i32, P(vp)], i32),
        "sg_plan_execute": ([vp, vp, vp, vp, vp], i32),
        "sg_plan_execute_grad": ([vp, vp, vp, vp, vp], i32),
        "sg_plan_get_info": ([vp, P(PlanInfo)], i32),
        "sg_plan_autotune": ([vp, vp, vp, vp], i32),
        "sg_plan_set_schedule": ([vp, i32, i32, i32, i32, i32], i32),
        "sg_plan_set_schedule_balanced": ([vp, i32, i32], i32),
        "sg_plan_destroy": ([vp], i32),
        "sg_integrate": ([vp, P(Problem), i32, vp, vp, vp, vp], i32),
        "sg_integrate_noalloc": ([vp, P(Problem), i32, vp, vp, vp, vp], i32),
        "sg_integrate_points": ([vp, P(Problem), vp, vp, vp, u64, vp], i32),
        "sg_version": ([], ctypes.c_char_p),
        "sg_context_save_tuning": ([vp, ctypes.c_char_p], i32),
        "sg_context_load_tuning": ([vp, ctypes.c_char_p, P(i32)], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    for name in ("sg_host_live_allocations", "sg_host_launches"):
        if hasattr(L, name):
            getattr(L, name).restype = ctypes.c_long
    if hasattr(L, "sg_host_fail_malloc_after"):
        L.sg_host_fail_malloc_after.argtypes = [ctypes.c_int]
        L.sg_host_fail_malloc_after.restype = None
    return L


def host_functions(L):
    """Results of the synchronous host functions (compared with the product
    library by the parent)."""
    out = {"status_strings": [L.sg_status_string(s).decode() for s in range(-1, 9)]}
    counts = []
    for d, q, rule in [(1, 1, 2), (1, 9, 1), (2, 5, 3), (3, 6, 2), (5, 13, 4), (10, 14, 5), (100, 108, 2),
                       (4096, 4102, 1), (1000, 1060, 2), (1000, 1061, 2), (40, 100, 3), (0, 1, 2), (3, 2, 2),
                       (3, 5, 9)]:
        a, b, c = u64(), u64(), u64()
        st = L.sg_counts(d, q, rule, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        counts.append([d, q, rule, st, a.value, b.value, c.value])
        L.sg_counts(d, q, rule, None, None, None)
    out["counts"] = counts
    rules = []
    for rule in range(0, 7):
        for level in (-1, 0, 1, 2, 3, 5, 8, 10, 17, 18):
            n = i32()
            st = L.sg_rule_table(rule, level, None, None, ctypes.byref(n))
            if st != 0 or level > 10:   # larger tables: the count only (Clenshaw-Curtis weights are O(n^2))
                rules.append([rule, level, st, n.value])
                continue
            x = np.zeros(n.value)
            w = np.zeros(n.value)
            st = L.sg_rule_table(rule, level, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(n))
            rules.append([rule, level, st, n.value, float(x.sum()), float(w.sum())])
    out["rules"] = rules
    coefs = []
    for d, q in [(1, 1), (5, 9), (60, 68), (100, 130), (200, 260)]:
        for e in range(-1, q - d + 2):
            c = i64()
            st = L.sg_coefficient(d, q, e, ctypes.byref(c))
            coefs.append([d, q, e, st, c.value])
    out["coefficients"] = coefs
    unr = []
    for d, q in [(1, 5), (3, 6), (5, 9), (7, 9)]:
        a = u64()
        L.sg_counts(d, q, 2, ctypes.byref(a), None, None)
        K = q - d
        for r in list(range(int(a.value))) + [int(a.value)]:
            coords = (i32 * max(K, 1))()
            levels = (i32 * max(K, 1))()
            nnz = i32()
            st = L.sg_unrank(d, q, r, coords, levels, ctypes.byref(nnz))
            unr.append([d, q, r, st] + ([nnz.value] + list(coords)[:nnz.value] + list(levels)[:nnz.value]
                                       if st == 0 else []))
    for d, q, r in [(1000, 1006, 0), (1000, 1006, 12345678901), (4096, 4100, 10 ** 12)]:
        coords = (i32 * 8)()
        levels = (i32 * 8)()
        nnz = i32()
        st = L.sg_unrank(d, q, r, coords, levels, ctypes.byref(nnz))
        unr.append([d, q, r, st, nnz.value] + list(coords)[:nnz.value] + list(levels)[:nnz.value])
    out["unrank"] = unr
    return out


def mixed_batch(seed, with_oscq=True):
    rng = np.random.default_rng(seed)
    probs = []
    off = 0
    dims = [1, 2, 3, 7, 63, 64, 65, 257, 1000, 4096, 5000]
    fams = [0, 1, 2, 4] + ([5, 6] if with_oscq else [])
    for i in range(40):
        d = int(dims[i % len(dims)])
        K = int(rng.integers(0, 9))
        rule = int(rng.integers(1, 6))
        fam = int(fams[i % len(fams)])
        probs.append((d, d + K, rule, fam, off))
        off += NPARAMS[fam](d)
    params = rng.uniform(0.05, 0.9, off)
    return probs, params


def problems_array(probs):
    arr = (Problem * len(probs))()
    for i, p in enumerate(probs):
        arr[i] = Problem(*p)
    return arr


def ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def plans(L, ctx, statuses):
    """Plans of mixed batches: build, execute (direct, graph), gradient,
    schedules, autotune, block variant; and the plan-free entry points."""
    fake_stream = ctypes.c_void_p(0x1000)
    for seed, with_oscq in [(0, True), (1, False)]:
        probs, params = mixed_batch(seed, with_oscq)
        arr = problems_array(probs)
        n = len(probs)
        for prec in (0, 1, 2):
            plan = vp()
            st = L.sg_plan_create(ctx, arr, n, prec, ctypes.byref(plan))
            statuses.append(["plan_create", seed, prec, st])
            if st != 0:
                continue
            info = PlanInfo()
            statuses.append(["get_info", L.sg_plan_get_info(plan, ctypes.byref(info))])
            statuses.append(["fp64_complex", info.fp64_complex, sum(1 for p in probs if p[3] in (5, 6))])
            outs = [np.zeros(n) for _ in range(10)]
            bound = np.zeros(n)
            grad = np.zeros(len(params))
            gout = np.ones(n)
            statuses.append(["execute", L.sg_plan_execute(plan, ptr(params), ptr(outs[0]), ptr(bound), None)])
            statuses.append(["execute_nobound", L.sg_plan_execute(plan, ptr(params), ptr(outs[0]), None, None)])
            statuses.append(["execute_grad", with_oscq,
                             L.sg_plan_execute_grad(plan, ptr(params), ptr(gout), ptr(grad), None)])
            for cpl, mg, cs, pers, gr in [(1, 1, 0, 0, 0), (4, 4, 1, 0, 1), (16, 2, 0, 1, 0), (64, 4, 1, 1, 1),
                                         (0, 1, 0, 0, 0), (65, 1, 0, 0, 0), (4, 3, 0, 0, 0), (4, 1, 2, 0, 0)]:
                statuses.append(["set_schedule", cpl, mg, cs, pers, gr,
                                 L.sg_plan_set_schedule(plan, cpl, mg, cs, pers, gr)])
                # graph replay bookkeeping: more bindings than the cache keeps
                for o in outs:
                    L.sg_plan_execute(plan, ptr(params), ptr(o), ptr(bound), fake_stream)
            for m, gr in [(1, 0), (2, 1), (4, 0), (8, 1), (0, 0), (9, 0), (2, 2)]:
                statuses.append(["balanced", m, gr, L.sg_plan_set_schedule_balanced(plan, m, gr)])
                L.sg_plan_execute(plan, ptr(params), ptr(outs[1]), ptr(bound), fake_stream)
            statuses.append(["autotune", L.sg_plan_autotune(plan, ptr(params), ptr(outs[2]), None)])
            statuses.append(["autotune_stream", L.sg_plan_autotune(plan, ptr(params), ptr(outs[2]), fake_stream)])
            statuses.append(["execute_after_tune",
                             L.sg_plan_execute(plan, ptr(params), ptr(outs[3]), ptr(bound), fake_stream)])
            statuses.append(["execute_null", L.sg_plan_execute(plan, None, ptr(outs[3]), None, None)])
            statuses.append(["destroy", L.sg_plan_destroy(plan)])
        # a second plan of the same classes reuses the autotune result
        plan = vp()
        statuses.append(["plan_reuse", L.sg_plan_create(ctx, arr, n, 0, ctypes.byref(plan))])
        L.sg_plan_destroy(plan)
        # block variant (no oscillatory-quadratic problems)
        bprobs = [p for p in probs if p[3] not in (5, 6)]
        barr = problems_array(bprobs)
        for m in (1, 2, 3, 10, 10000, 0):
            plan = vp()
            st = L.sg_plan_create_blocked(ctx, barr, len(bprobs), 1, m, ctypes.byref(plan))
            statuses.append(["blocked", seed, m, st])
            if st == 0:
                out = np.zeros(len(bprobs))
                bound = np.zeros(len(bprobs))
                statuses.append(["blocked_exec", L.sg_plan_execute(plan, ptr(params), ptr(out), ptr(bound),
                                                                  fake_stream)])
                statuses.append(["blocked_exec2", L.sg_plan_execute(plan, ptr(params), ptr(out), None, None)])
                statuses.append(["blocked_tune", L.sg_plan_autotune(plan, ptr(params), ptr(out), fake_stream)])
                statuses.append(["blocked_grad", L.sg_plan_execute_grad(plan, ptr(params), ptr(out), ptr(out),
                                                                       None)])
                L.sg_plan_destroy(plan)
        if with_oscq:
            plan = vp()
            st = L.sg_plan_create_blocked(ctx, arr, n, 1, 2, ctypes.byref(plan))
            statuses.append(["blocked_oscq", st])
            if st == 0:
                info = PlanInfo()
                L.sg_plan_get_info(plan, ctypes.byref(info))
                statuses.append(["fp64_complex", info.fp64_complex, sum(1 for p in probs if p[3] in (5, 6))])
                # block sub-problems: one per block (two for the complex-sweep
                # families), so the units are sum d, or 2 d for those
                statuses.append(["blocked_units", int(info.units),
                                 sum(p[0] * (2 if p[3] in (5, 6) else 1) for p in probs)])
                L.sg_plan_destroy(plan)
    # rejected plans
    for bad in [[(0, 1, 2, 0, 0)], [(3, 2, 2, 0, 0)], [(3, 5, 9, 0, 0)], [(3, 5, 2, 9, 0)], [(3, 12, 2, 0, 0)],
                [(3, 5, 2, 3, 0)], [(3, 5, 2, 0, -1)]]:
        plan = vp()
        statuses.append(["bad_plan", bad[0], L.sg_plan_create(ctx, problems_array(bad), 1, 0, ctypes.byref(plan))])
    plan = vp()
    statuses.append(["bad_prec", L.sg_plan_create(ctx, problems_array([(3, 5, 2, 0, 0)]), 1, 7,
                                                  ctypes.byref(plan))])
    statuses.append(["bad_n", L.sg_plan_create(ctx, problems_array([(3, 5, 2, 0, 0)]), 0, 0, ctypes.byref(plan))])
    # plan-free entry points
    rng = np.random.default_rng(5)
    for d in (1, 255, 256, 257, 4096, 70000, 262144, 300000):
        for fam in (0, 1, 2, 4, 5, 6):
            for K in (0, 3, 8, 9):
                params = rng.uniform(0.05, 0.5, NPARAMS[fam](d))
                out = np.zeros(1)
                bound = np.zeros(1)
                pr = Problem(d, d + K, 2, fam, 0)
                for prec in (0, 1):
                    statuses.append(["integrate", d, fam, K, prec,
                                     L.sg_integrate(ctx, ctypes.byref(pr), prec, ptr(params), ptr(out), ptr(bound),
                                                    None)])
                    statuses.append(["noalloc", d, fam, K, prec,
                                     L.sg_integrate_noalloc(ctx, ctypes.byref(pr), prec, ptr(params), ptr(out),
                                                            None, None)])
    for d, K in [(1, 0), (3, 4), (10, 3), (40, 5)]:
        for fam in range(7):
            params = rng.uniform(0.05, 0.5, NPARAMS[fam](d))
            out = np.zeros(1)
            bound = np.zeros(1)
            pr = Problem(d, d + K, 3, fam, 0)
            statuses.append(["points", d, K, fam,
                             L.sg_integrate_points(ctx, ctypes.byref(pr), ptr(params), ptr(out), ptr(bound),
                                                   10 ** 7, None)])
    # device unranking
    coords = np.zeros((1000, 8), np.int32)
    levels = np.zeros((1000, 8), np.int32)
    nnz = np.zeros(1000, np.int32)
    for d, q, r0, cnt, mx in [(5, 9, 0, 100, 4), (50, 56, 1000, 1000, 8), (5, 9, 120, 10, 4), (5, 9, 0, 10, 3)]:
        statuses.append(["unrank_device", d, q, r0, cnt, mx,
                         L.sg_unrank_device(ctx, d, q, r0, cnt, mx, ptr(coords), ptr(levels), ptr(nnz), None)])
    statuses.append(["last_error", L.sg_last_error(ctx).decode()[:200]])


def fail_malloc_scan(L):
    """A context, plans and plan-free calls with the n-th allocation failing,
    for n = 1, 2, ... until the whole sequence succeeds.  For every n and
    call: the status, the launches the call made and, after everything is
    destroyed, the allocations still alive."""
    probs, params = mixed_batch(0, True)
    bprobs = [p for p in probs if p[3] not in (5, 6)]
    p1 = np.full(4096, 0.1)
    out = np.zeros(len(probs))
    rows = []
    for n in range(1, 400):
        L.sg_host_fail_malloc_after(n)
        calls = []

        def call(name, f):
            l0 = L.sg_host_launches()
            st = f()
            calls.append([name, st, L.sg_host_launches() - l0])
            return st

        ctx = vp()
        if call("context", lambda: L.sg_context_create(ctypes.byref(ctx))) == 0:
            plan = vp()
            if call("plan", lambda: L.sg_plan_create(ctx, problems_array(probs), len(probs), 1,
                                                     ctypes.byref(plan))) == 0:
                call("balanced", lambda: L.sg_plan_set_schedule_balanced(plan, 2, 0))
                call("schedule", lambda: L.sg_plan_set_schedule(plan, 4, 4, 1, 1, 0))
                call("autotune", lambda: L.sg_plan_autotune(plan, ptr(params), ptr(out), None))
                call("execute", lambda: L.sg_plan_execute(plan, ptr(params), ptr(out), None, None))
                L.sg_plan_destroy(plan)
            plan = vp()
            if call("blocked", lambda: L.sg_plan_create_blocked(ctx, problems_array(bprobs), len(bprobs), 0, 3,
                                                                ctypes.byref(plan))) == 0:
                call("blocked_execute", lambda: L.sg_plan_execute(plan, ptr(params), ptr(out), None, None))
                L.sg_plan_destroy(plan)
            pr = Problem(4096, 4100, 2, 0, 0)
            call("integrate", lambda: L.sg_integrate(ctx, ctypes.byref(pr), 0, ptr(p1), ptr(out), None, None))
            pr2 = Problem(10, 13, 2, 0, 0)
            call("points", lambda: L.sg_integrate_points(ctx, ctypes.byref(pr2), ptr(p1), ptr(out), None, 0,
                                                         None))
            L.sg_context_destroy(ctx)
        L.sg_host_fail_malloc_after(0)
        rows.append([n, calls, L.sg_host_live_allocations()])
        if all(c[1] == 0 for c in calls):
            break
    return rows


def tuning(L, tmpdir):
    """Autotune records: reuse only by plans of the same shape, saved and
    loaded across contexts, ignored for another device, and a reader that
    survives malformed files."""
    import random
    res = {"version": L.sg_version().decode()}
    probs, params = mixed_batch(0, True)
    other, _ = mixed_batch(1, False)
    shuffled = list(reversed(probs))
    out = np.zeros(len(probs))

    def info_of(ctx, pr):
        plan = vp()
        st = L.sg_plan_create(ctx, problems_array(pr), len(pr), 1, ctypes.byref(plan))
        assert st == 0
        info = PlanInfo()
        L.sg_plan_get_info(plan, ctypes.byref(info))
        L.sg_plan_destroy(plan)
        return [info.coords_per_lane, info.max_group, info.balanced, info.persistent, info.cost_scaled]

    ctx = vp()
    L.sg_context_create(ctypes.byref(ctx))
    res["default"] = info_of(ctx, probs)
    plan = vp()
    L.sg_plan_create(ctx, problems_array(probs), len(probs), 1, ctypes.byref(plan))
    res["autotune"] = L.sg_plan_autotune(plan, ptr(params), ptr(out), None)
    info = PlanInfo()
    L.sg_plan_get_info(plan, ctypes.byref(info))
    res["tuned"] = [info.coords_per_lane, info.max_group, info.balanced, info.persistent, info.cost_scaled]
    L.sg_plan_destroy(plan)
    res["same_shape_permuted"] = info_of(ctx, shuffled)
    res["other_shape"] = info_of(ctx, other)
    path = os.path.join(tmpdir, "tune.json").encode()
    res["save"] = L.sg_context_save_tuning(ctx, path)
    res["save_null"] = L.sg_context_save_tuning(ctx, None)
    res["save_bad_dir"] = L.sg_context_save_tuning(ctx, os.path.join(tmpdir, "no", "such", "dir.json").encode())
    L.sg_context_destroy(ctx)
    text = open(path, "rb").read()
    res["text"] = text.decode()

    ctx = vp()
    L.sg_context_create(ctypes.byref(ctx))
    n = i32(-1)
    res["load"] = [L.sg_context_load_tuning(ctx, path, ctypes.byref(n)), n.value]
    res["loaded_shape"] = info_of(ctx, probs)
    res["load_missing"] = L.sg_context_load_tuning(ctx, os.path.join(tmpdir, "missing.json").encode(), None)
    L.sg_context_destroy(ctx)

    # another device or version: nothing loaded
    ctx = vp()
    L.sg_context_create(ctypes.byref(ctx))
    foreign = []
    for old, new in [(b'"arch": "host-stand-in"', b'"arch": "gfx942"'), (b'"compute_units": 256', b'"compute_units": 304'),
                     (b'"version": "' + res["version"].encode() + b'"', b'"version": "0.0.1"')]:
        pth = os.path.join(tmpdir, "foreign.json").encode()
        open(pth, "wb").write(text.replace(old, new))
        n = i32(-1)
        foreign.append([L.sg_context_load_tuning(ctx, pth, ctypes.byref(n)), n.value])
    res["foreign"] = foreign
    res["foreign_shape"] = info_of(ctx, probs)

    # malformed files: every load returns OK or INVALID_ARGUMENT, and a
    # rejected file loads nothing
    rnd = random.Random(7)
    codes = []
    pth = os.path.join(tmpdir, "fuzz.json").encode()
    cases = [b"", b"{", b"[" * 100000, b"{" * 100000, b'{"format": "sgmdi-autotune-1"}', b"null", b"123",
             b'{"a": "\\u0041"}', text + b"x", text[:-3], text.replace(b"1", b"99999999999999999999"),
             text.replace(b'"balanced": 0', b'"balanced": 9'), text.replace(b'"max_group": 1', b'"max_group": 3'),
             text.replace(b"[", b"{", 1), text.replace(b'"key"', b'"kee"')]
    for _ in range(400):
        b = bytearray(text)
        for _ in range(rnd.randint(1, 4)):
            op = rnd.randrange(4)
            pos = rnd.randrange(len(b)) if b else 0
            if op == 0 and b:
                b[pos] = rnd.randrange(256)
            elif op == 1 and b:
                del b[pos]
            elif op == 2:
                b[pos:pos] = bytes([rnd.choice(b'{}[],:"0123456789-eE.tn\\ ')])
            else:
                b = b[:pos]
        cases.append(bytes(b))
    for c in cases:
        open(pth, "wb").write(c)
        n = i32(-1)
        st = L.sg_context_load_tuning(ctx, pth, ctypes.byref(n))
        codes.append([st, n.value])
    res["fuzz"] = codes
    L.sg_context_destroy(ctx)
    return res


def main():
    path = sys.argv[1]
    L = load(path)
    res = {}
    if "--tuning" in sys.argv:
        res["tuning"] = tuning(L, sys.argv[sys.argv.index("--tuning") + 1])
        res["live"] = L.sg_host_live_allocations()
        print(json.dumps(res))
        return
    if "--fail-malloc" in sys.argv:
        res["fail_malloc"] = fail_malloc_scan(L)
        res["live"] = L.sg_host_live_allocations()
        print(json.dumps(res))
        return
    res["host"] = host_functions(L)
    statuses = []
    ctx = vp()
    st = L.sg_context_create(ctypes.byref(ctx))
    statuses.append(["context", st])
    statuses.append(["context_null", L.sg_context_create(None)])
    if st == 0:
        plans(L, ctx, statuses)
        L.sg_context_destroy(ctx)
    L.sg_context_destroy(None)
    L.sg_plan_destroy(None)
    res["statuses"] = statuses
    res["live"] = L.sg_host_live_allocations()
    res["launches"] = L.sg_host_launches()
    if "--oracle" in sys.argv:
        import oracle
        oracle._lib = oracle.load(oracle.SAN_LIB_PATH)
        orc = {}
        orc["rules"] = [[r, lv, float(np.sum(oracle.rule(r, lv)[1]))] for r in ("tr", "cc", "gp", "gl", "gl_paper")
                        for lv in (1, 2, 4, 7)]
        total, coords, levels, nnz = oracle.enumerate_window(4, 8)
        orc["enumerate"] = [total, int(nnz.sum()), int(levels.sum())]
        rng = np.random.default_rng(3)
        vals = []
        for fam in ("exp_sum", "oscillatory", "product_peak", "gaussian", "oscillatory_quadratic", "corner_peak",
                    "oscillatory_quadratic_linear"):
            d = 4
            k = {"exp_sum": d, "oscillatory": d + 1, "product_peak": 2 * d, "gaussian": 2 * d,
                 "oscillatory_quadratic": 2 * d + 1, "corner_peak": d, "oscillatory_quadratic_linear": 3 * d + 1}[fam]
            p = rng.uniform(0.1, 0.6, k)
            vals.append([fam, oracle.smolyak_points(4, 7, "cc", fam, p, nthreads=2)["q"]])
            if fam != "corner_peak":
                vals.append([fam, oracle.smolyak_factorised(4, 7, "gp", fam, p)])
                vals.append([fam, list(oracle.smolyak_factorised_hilo(4, 7, "gl", fam, p))])
            if fam not in ("corner_peak", "oscillatory_quadratic"):
                g = oracle.smolyak_factorised_grad(4, 9, "cc", fam, p)
                vals.append([fam, [float(v) for v in g]])
        orc["values"] = vals
        res["oracle"] = orc
    print(json.dumps(res))


if __name__ == "__main__":
    main()
