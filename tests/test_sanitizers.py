"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The runtime's host logic (the C ABI: validation, counts, rule tables,
unranking, plan building, schedules, graph bookkeeping, autotune, the
plan-free entry points) is compiled with the host compiler and the
sanitizers, against a host stand-in for the HIP runtime whose "device"
memory is host heap, so every upload is checked against its allocation;
the oracle is compiled the same way.  Both run in a child process that
preloads the ASan runtime (tests/sanitized_host_run.py): any sanitizer
report aborts it.  The host results must equal the product library's, and
with every allocation failing in turn, each call must report OUT_OF_MEMORY,
launch nothing and leave no allocation behind.
"""
from __future__ import annotations

import glob
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2210_14313_amd import build as B  # noqa: E402
import oracle  # noqa: E402

RUNNER = os.path.join(ROOT, "tests", "sanitized_host_run.py")
OK, INVALID, UNSUPPORTED, OVERFLOW, OOM = 0, 1, 2, 3, 4


def _stale(lib, sources):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    return any(os.path.getmtime(s) > t for s in sources)


def _asan_runtime():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip("the ASan runtime of the host compiler is not installed")
    return path


@pytest.fixture(scope="module")
def sanitized():
    srcs = (glob.glob(os.path.join(B.CSRC, "*.cpp")) + glob.glob(os.path.join(B.CSRC, "*.hpp")) +
            glob.glob(os.path.join(ROOT, "include", "*.h")))
    if _stale(B.HOSTSAN_LIB, srcs):
        B.build_host_sanitized()
    if _stale(oracle.SAN_LIB_PATH, [oracle.SRC_PATH]):
        oracle.build_sanitized()
    return B.HOSTSAN_LIB


def _run(lib, *flags):
    env = dict(os.environ)
    env["LD_PRELOAD"] = _asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env.pop("SGMDI_LIB", None)
    r = subprocess.run([sys.executable, RUNNER, lib, *flags], capture_output=True, text=True, env=env,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    for marker in ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer"):
        assert marker not in r.stderr, r.stderr[-4000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


@pytest.fixture(scope="module")
def run_result(sanitized):
    return _run(sanitized, "--oracle")


def test_host_results_match_product_library(run_result):
    """The sanitized build computes the same host results as libsgmdi.so."""
    import sanitized_host_run as R
    L = R.load(os.path.join(ROOT, "paper_2210_14313_amd", "libsgmdi.so"))
    ref = R.host_functions(L)
    got = run_result["host"]
    for key in ("status_strings", "counts", "coefficients", "unrank"):
        assert got[key] == ref[key], key
    assert len(got["rules"]) == len(ref["rules"])
    for a, b in zip(got["rules"], ref["rules"]):
        assert a[:4] == b[:4]
        if len(a) > 4:
            np.testing.assert_allclose(a[4:], b[4:], rtol=1e-14)


def test_plan_paths_statuses(run_result):
    """Every plan and plan-free call of the sanitized host run returns what the header
    documents, and nothing is left allocated."""
    st = run_result["statuses"]
    assert ["context", OK] in st and ["context_null", INVALID] in st
    by = {}
    for s in st:
        by.setdefault(s[0], []).append(s)
    assert all(s[-1] == OK for s in by["plan_create"]) and len(by["plan_create"]) == 6
    assert all(s[-1] == OK for k in ("get_info", "execute", "execute_nobound", "autotune", "autotune_stream",
                                    "execute_after_tune", "destroy", "plan_reuse") for s in by[k])
    assert all(s[-1] == INVALID for s in by["execute_null"])
    # gradient: every family, the oscillatory quadratic by its complex reverse sweep
    assert all(s[2] == OK for s in by["execute_grad"])
    for s in by["set_schedule"]:
        _, cpl, mg, cs, pers, gr, code = s
        valid = 1 <= cpl <= 64 and mg in (1, 2, 4) and cs in (0, 1)
        assert code == (OK if valid else INVALID), s
    for _, m, gr, code in by["balanced"]:
        assert code == (OK if 1 <= m <= 8 and gr in (0, 1) else INVALID)
    for _, seed, m, code in by["blocked"]:
        assert code == (OK if m >= 1 else INVALID)
    assert all(s[-1] == OK for k in ("blocked_exec", "blocked_exec2", "blocked_tune") for s in by[k])
    assert all(s[-1] == UNSUPPORTED for s in by["blocked_grad"])
    bad = {tuple(s[1]): s[2] for s in by["bad_plan"]}
    assert bad[(0, 1, 2, 0, 0)] == INVALID and bad[(3, 2, 2, 0, 0)] == INVALID
    assert bad[(3, 5, 9, 0, 0)] == INVALID and bad[(3, 5, 2, 9, 0)] == INVALID
    assert bad[(3, 12, 2, 0, 0)] == UNSUPPORTED and bad[(3, 5, 2, 3, 0)] == UNSUPPORTED
    assert bad[(3, 5, 2, 0, -1)] == INVALID
    assert by["bad_prec"][0][-1] == INVALID and by["bad_n"][0][-1] == INVALID
    for _, d, fam, K, prec, code in by["integrate"] + by["noalloc"]:
        assert code == (UNSUPPORTED if K > 8 else OK), (d, fam, K, prec, code)
    from paper_2210_14313_amd import native
    for _, d, K, fam, code in by["points"]:
        npts = native.counts(d, d + K, "gp")[1]
        assert code == (OK if npts <= 10 ** 7 else UNSUPPORTED), (d, K, fam, code)
    ud = {tuple(s[1:6]): s[6] for s in by["unrank_device"]}
    assert ud[(5, 9, 0, 100, 4)] == OK and ud[(50, 56, 1000, 1000, 8)] == OK
    assert ud[(5, 9, 120, 10, 4)] == INVALID and ud[(5, 9, 0, 10, 3)] == INVALID
    # oscillatory-quadratic integrands run in FP64 in every mode, and the plan says how many
    assert len(by["fp64_complex"]) == 7
    assert all(got == want for _, got, want in by["fp64_complex"])
    assert any(want > 0 for _, got, want in by["fp64_complex"])
    # block plans sweep an oscillatory block once (its phase cancelled), a
    # complex-sweep block twice
    assert by["blocked_units"] and all(got == want for _, got, want in by["blocked_units"])
    assert run_result["live"] == 0


def test_oracle_under_sanitizers(run_result):
    """The sanitized oracle gives the same values as the product build of it."""
    orc = run_result["oracle"]
    total, coords, levels, nnz = oracle.enumerate_window(4, 8)
    assert orc["enumerate"] == [total, int(nnz.sum()), int(levels.sum())]
    for r, lv, wsum in orc["rules"]:
        assert wsum == pytest.approx(float(np.sum(oracle.rule(r, lv)[1])), rel=1e-15)
    rng = np.random.default_rng(3)
    vals = iter(orc["values"])
    for fam in ("exp_sum", "oscillatory", "product_peak", "gaussian", "oscillatory_quadratic", "corner_peak",
                "oscillatory_quadratic_linear"):
        k = {"exp_sum": 4, "oscillatory": 5, "product_peak": 8, "gaussian": 8, "oscillatory_quadratic": 9,
             "corner_peak": 4, "oscillatory_quadratic_linear": 13}[fam]
        p = rng.uniform(0.1, 0.6, k)
        assert next(vals)[1] == pytest.approx(oracle.smolyak_points(4, 7, "cc", fam, p, nthreads=2)["q"],
                                              rel=1e-15, abs=1e-300)
        if fam != "corner_peak":
            assert next(vals)[1] == oracle.smolyak_factorised(4, 7, "gp", fam, p)
            assert tuple(next(vals)[1]) == oracle.smolyak_factorised_hilo(4, 7, "gl", fam, p)
        if fam not in ("corner_peak", "oscillatory_quadratic"):
            np.testing.assert_array_equal(next(vals)[1], oracle.smolyak_factorised_grad(4, 9, "cc", fam, p))


def test_allocation_failures(sanitized):
    """With the n-th device allocation failing (n = 1, 2, ...), the call that
    makes it reports OUT_OF_MEMORY and launches nothing, every other call
    succeeds, and destroying everything leaves no allocation alive."""
    res = _run(sanitized, "--fail-malloc")
    rows = res["fail_malloc"]
    assert len(rows) > 5
    failed_calls = set()
    for n, calls, live in rows:
        assert live == 0, (n, calls)
        failing = [c for c in calls if c[1] != OK]
        if n < rows[-1][0]:
            assert len(failing) == 1, (n, calls)
        for name, code, launches in failing:
            assert code == OOM and launches == 0, (n, name, code, launches)
            failed_calls.add(name)
    assert all(c[1] == OK for c in rows[-1][1])
    assert {"plan", "blocked", "integrate", "points"} <= failed_calls
    assert res["live"] == 0


def test_autotune_records_on_disk(sanitized, tmp_path):
    """Tuned schedules are reused only by plans of the same shape (the
    sorted (d, K, rule, family) list), survive a save and load into a new
    context, are ignored when written for another device or version, and a
    malformed file is rejected whole without a sanitizer report."""
    r = _run(sanitized, "--tuning", str(tmp_path))["tuning"]
    default, tuned = r["default"], r["tuned"]
    assert r["autotune"] == OK and tuned != default
    assert r["same_shape_permuted"] == tuned      # order of the problems does not matter
    assert r["other_shape"] == default            # same count, other classes: not inherited
    assert r["save"] == OK and r["save_null"] == INVALID and r["save_bad_dir"] == INVALID
    doc = json.loads(r["text"])
    assert doc["version"] == r["version"] and doc["compute_units"] == 256 and len(doc["entries"]) == 1
    assert r["load"] == [OK, 1] and r["loaded_shape"] == tuned
    assert r["load_missing"] == INVALID
    assert r["foreign"] == [[OK, 0]] * 3 and r["foreign_shape"] == default
    codes = r["fuzz"]
    assert all(st in (OK, INVALID) for st, n in codes)
    assert all(n == 0 for st, n in codes if st == INVALID)
    assert all(n in (0, 1) for st, n in codes)
    assert codes[:10] == [[INVALID, 0]] * 10
