"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances: FP64 mode within 1e-12 relative; the FP32-compensated mode
within the a-priori bound the library states for every result, and within
1e-7 relative on the standard workloads.  "Relative" is against the oracle's
accuracy scale (oracle.accuracy_scale): |Q|, and for the oscillatory family
the modulus |S| = sqrt(Q(w)^2 + Q(w - 1/4)^2) of the complex Smolyak sum
whose real part Q is (Q itself passes through zero as w varies).
"""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module")
def api(torch_dev):
    from paper_2210_14313_amd import api as A, native
    native.lib()
    return A


def _scale(batch, ref):
    import oracle
    return oracle.accuracy_scale(batch, ref)


def _run(api, batch, precision, with_bound=True):
    vals, bnd = api.integrate(batch, precision, with_bound=with_bound)
    return vals.cpu().numpy(), (bnd.cpu().numpy() if bnd is not None else None)


def _point_ref(orc, batch):
    return np.array([orc.smolyak_points(p.d, p.q, p.rule, p.family, batch.param_slice(i))["q"]
                     for i, p in enumerate(batch.problems)])


def _fact_ref(orc, batch):
    return orc.batch_factorised(batch)


# ---------------------------------------------------------------- small
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_small_random_batches_fp64(api, orc, seed):
    from paper_2210_14313_amd import workloads as W
    b = W.random_small(seed, 64, d_range=(1, 12), k_range=(0, 5))
    say("case small_random fp64 seed", seed)
    got, bnd = _run(api, b, "fp64")
    ref = _point_ref(orc, b)
    err = np.abs(got - ref) / _scale(b, ref)
    assert np.max(err) <= 1e-12, (np.argmax(err), np.max(err))
    assert np.all(np.abs(got - ref) <= bnd + 1e-300)


@pytest.mark.parametrize("prec", ["fp32c", "fp32e"])
@pytest.mark.parametrize("seed", [1, 2])
def test_small_random_batches_fp32(api, orc, seed, prec):
    from paper_2210_14313_amd import workloads as W
    b = W.random_small(seed, 64, d_range=(1, 12), k_range=(0, 5))
    say("case small_random", prec, "seed", seed)
    got, bnd = _run(api, b, prec)
    ref = _point_ref(orc, b)
    assert np.all(np.abs(got - ref) <= bnd), np.max(np.abs(got - ref) / bnd)
    # the 1e-7 target is stated for the oscillatory and exp-sum families
    sel = np.array([p.family != "product_peak" for p in b.problems])
    assert np.max((np.abs(got - ref) / _scale(b, ref))[sel]) <= 1e-7


@pytest.mark.parametrize("prec", ["fp32c", "fp32e"])
def test_product_peak_fp32_accuracy(api, orc, prec):
    """The product-peak family in the FP32 modes (its pair values are FP64
    values rounded once; the 1e-7 target is stated for the oscillatory and
    exp-sum families only): within the bound, and within 1e-4 of |Q| on
    random small integrands of every rule (measured 1.2e-5 / 4.4e-6), 1e-6
    at d = 64-256 (measured up to 2.5e-7)."""
    from paper_2210_14313_amd import workloads as W
    for seed in (501, 502, 503, 504):
        b = W.random_small(seed, 64, d_range=(1, 40), k_range=(0, 6), families=("product_peak",),
                           rules=W.ALL_RULES)
        say("case product-peak fp32", prec, seed)
        ref = _fact_ref(orc, b)
        got, bnd = _run(api, b, prec)
        assert np.all(np.abs(got - ref) <= bnd), np.max(np.abs(got - ref) / bnd)
        assert np.max(np.abs(got - ref) / np.abs(ref)) <= 1e-4
    rng = np.random.default_rng(77)
    for d, K, rule in [(100, 5, "cc"), (256, 4, "gl"), (200, 6, "gp"), (64, 8, "cc")]:
        b = W.single(d, d + K, rule, "product_peak", W.draw_params(rng, "product_peak", d))
        say("case product-peak fp32 large", prec, d, K, rule)
        ref = _fact_ref(orc, b)
        got, bnd = _run(api, b, prec)
        assert abs(got[0] - ref[0]) <= bnd[0]
        assert abs(got[0] - ref[0]) <= 1e-6 * abs(ref[0]), (d, K, rule, got[0], ref[0])


# -------------------------------------------- several tiles, ragged tails
TILE_CASES = [(63, 2, "cc", "exp_sum"), (64, 3, "gl", "oscillatory"), (65, 2, "tr", "product_peak"),
              (255, 2, "cc", "oscillatory"), (257, 2, "gl", "exp_sum"), (300, 2, "cc", "product_peak"),
              (513, 1, "tr", "exp_sum"), (40, 8, "cc", "exp_sum"), (20, 8, "gl", "oscillatory"),
              (1, 8, "cc", "exp_sum"), (1, 0, "gl", "oscillatory"), (7, 0, "cc", "product_peak"),
              (2, 8, "gl_paper", "product_peak"), (129, 3, "gl_paper", "exp_sum")]


@pytest.mark.parametrize("d,K,rule,family", TILE_CASES)
def test_tiles_and_edges(api, orc, d, K, rule, family):
    from paper_2210_14313_amd import workloads as W
    rng = np.random.default_rng(d * 1000 + K)
    b = W.single(d, d + K, rule, family, W.draw_params(rng, family, d))
    say("case tile", d, K, rule, family)
    npts = orc.counts.counts_by_generating_function(d, d + K, rule)["n_points_rep"]
    ref = _point_ref(orc, b) if npts <= 3e8 else _fact_ref(orc, b)
    tol32 = 1e-7 if family != "product_peak" else 1.0
    for prec, tol in (("fp64", 1e-12), ("fp32c", tol32), ("fp32e", tol32)):
        got, bnd = _run(api, b, prec)
        err = np.abs(got - ref) / _scale(b, ref)
        assert err[0] <= tol, (prec, got, ref, err)
        assert np.abs(got - ref)[0] <= bnd[0], (prec, got, ref, bnd)


def test_large_arguments_take_the_exact_branch(api, orc):
    # |parameter * y| > 1/2 switches from the series to expm1 / sin
    from paper_2210_14313_amd import workloads as W
    for fam, params in (("exp_sum", np.array([3.0, -2.5, 0.2, 6.0])),
                        ("oscillatory", np.array([0.3, 7.0, -3.0, 1.5, 12.0]))):
        b = W.single(4, 9, "cc", fam, params)
        say("case large-arguments", fam)
        ref = _point_ref(orc, b)
        got, bnd = _run(api, b, "fp64")
        assert abs(got[0] - ref[0]) <= 1e-12 * _scale(b, ref)[0]
        for prec in ("fp32c", "fp32e"):
            got, bnd = _run(api, b, prec)
            assert abs(got[0] - ref[0]) <= bnd[0], prec


# ---------------------------------------------------------- full sizes
def test_plain_exp_d10_full(api, orc):
    from paper_2210_14313_amd import workloads as W
    b = W.plain_exp_d10()
    say("case plain_exp_d10 full")
    ref = _point_ref(orc, b)
    got, _ = _run(api, b, "fp64")
    assert abs(got[0] - ref[0]) <= 1e-12 * abs(ref[0])
    for prec in ("fp32c", "fp32e"):
        got32, bnd = _run(api, b, prec)
        assert abs(got32[0] - ref[0]) <= bnd[0], prec


def _golden_rows():
    path = os.path.join(GOLDEN, "oracle_full_size.json")
    if not os.path.exists(path):
        return []
    return json.load(open(path))["rows"]


@pytest.mark.parametrize("row", _golden_rows(), ids=lambda r: f"{r['workload']}-{r['index']}")
def test_full_size_against_stored_point_oracle(api, orc, row):
    from paper_2210_14313_amd import workloads as W
    batch = W.STANDARD[row["workload"]]()
    b = batch.subset([row["index"]])
    p = b.problems[0]
    assert (p.d, p.q, p.rule, p.family) == (row["d"], row["q"], row["rule"], row["family"])
    ref = row["points_hi"] + row["points_lo"]
    say("case full-size", row["workload"], row["index"], p.family, p.rule)
    got, _ = _run(api, b, "fp64")
    scale = orc.accuracy_scale_one(p.d, p.q, p.rule, p.family, b.param_slice(0), ref)
    assert abs(got[0] - ref) <= 1e-12 * scale, (got, ref)
    for prec in ("fp32c", "fp32e"):
        got32, bnd = _run(api, b, prec)
        assert abs(got32[0] - ref) <= bnd[0], prec
        if p.family != "product_peak":
            assert abs(got32[0] - ref) <= 1e-7 * scale, prec


def test_batched_uneven_full_launch(api, orc):
    """The 4096-integrand batch in the launch configuration the benchmark
    times: every result against the binary128 oracle, and a sample of the
    cheaper integrands against the point-by-point oracle."""
    import torch
    from paper_2210_14313_amd import native, workloads as W
    b = W.batched_uneven()
    params = api.params_tensor(b)
    ref = _fact_ref(orc, b)
    scale = _scale(b, ref)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    for prec, tol in (("fp64", 1e-12), ("fp32c", 1e-7), ("fp32e", 1e-7)):
        say("case batched_uneven", prec)
        plan = native.Plan(b.problems, prec)
        plan.set_schedule(3, 4, graph=True)
        out = torch.empty(len(b), dtype=torch.float64, device="cuda")
        bnd = torch.empty_like(out)
        with torch.cuda.stream(stream):
            plan.execute(params, out, bnd, stream=stream)     # captured graph
            plan.execute(params, out, bnd, stream=stream)     # replay
        stream.synchronize()
        got, bd = out.cpu().numpy(), bnd.cpu().numpy()
        err = np.abs(got - ref) / scale
        assert np.max(err) <= tol, (prec, int(np.argmax(err)), float(np.max(err)))
        assert np.all(np.abs(got - ref) <= bd), prec
        plan.close()
    # sampled integrands against the point oracle
    npts = np.array([orc.counts.counts_by_generating_function(p.d, p.q, p.rule)["n_points_rep"]
                     for p in b.problems])
    idx = [int(i) for i in np.nonzero(npts <= 2e7)[0][:24]]
    assert len(idx) >= 8
    sub = b.subset(idx)
    pref = _point_ref(orc, sub)
    got, _ = _run(api, sub, "fp64")
    assert np.max(np.abs(got - pref) / _scale(sub, pref)) <= 1e-12


def test_gradient_workload_forward(api, orc):
    from paper_2210_14313_amd import workloads as W
    b = W.gradient_osc_d200()
    say("case gradient_osc_d200 forward")
    ref = _fact_ref(orc, b)
    got, _ = _run(api, b, "fp64")
    assert np.max(np.abs(got - ref) / _scale(b, ref)) <= 1e-12


# -------------------------------------------------- determinism and paths
def test_determinism_graph_and_plain_path(api, orc):
    import torch
    from paper_2210_14313_amd import native, workloads as W
    b = W.random_small(9, 100, d_range=(1, 300), k_range=(0, 6))
    params = api.params_tensor(b)
    say("case determinism")
    for prec, pq in (("fp64", False), ("fp32c", True), ("fp32e", False)):
        plan = native.Plan(b.problems, prec)
        plan.set_schedule(2, 4, graph=True, persistent=pq)
        a = plan.execute(params).clone()           # default stream: no graph
        c = plan.execute(params).clone()
        assert torch.equal(a, c)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        outs = []
        for _ in range(3):                         # capture, then replays
            o = torch.empty_like(a)
            s.wait_stream(torch.cuda.current_stream())
            plan.execute(params, o, stream=s)
            s.synchronize()
            outs.append(o)
        o = torch.empty_like(a)
        s.wait_stream(torch.cuda.current_stream())
        for _ in range(3):
            plan.execute(params, o, stream=s)
            s.synchronize()
            assert torch.equal(o, a)
        for o in outs:
            assert torch.equal(o, a)
        plan.close()
        # plain single-integrand path
        for i in range(0, len(b), 17):
            p = b.problems[i]
            pi = torch.as_tensor(b.param_slice(i)).cuda()
            v = native.integrate_one(p, pi, prec).item()
            assert abs(v - a[i].item()) <= 1e-14 * max(abs(a[i].item()), 1.0)


def test_parameter_update_between_replays(api, orc):
    import torch
    from paper_2210_14313_amd import native, workloads as W
    b = W.random_small(10, 32, d_range=(2, 40), k_range=(1, 5))
    params = api.params_tensor(b)
    plan = native.Plan(b.problems, "fp64")
    s = torch.cuda.Stream()
    out = torch.empty(len(b), dtype=torch.float64, device="cuda")
    s.wait_stream(torch.cuda.current_stream())
    plan.execute(params, out, stream=s)
    s.synchronize()
    say("case parameter update")
    rng = np.random.default_rng(11)
    b2 = W.concat([W.single(p.d, p.q, p.rule, p.family, W.draw_params(rng, p.family, p.d))
                   for p in b.problems])
    assert len(b2.params) == len(b.params)
    params.copy_(torch.as_tensor(b2.params))
    s.wait_stream(torch.cuda.current_stream())
    plan.execute(params, out, stream=s)            # replay with new values
    s.synchronize()
    ref = _point_ref(orc, b2)
    got = out.cpu().numpy()
    assert np.max(np.abs(got - ref) / _scale(b2, ref)) <= 1e-12
    plan.close()


# ------------------------------------------------------------ unranking
@pytest.mark.parametrize("d,q", [(1, 5), (3, 7), (6, 10), (9, 11), (12, 12)])
def test_unrank_device_bit_exact(api, orc, d, q):
    from paper_2210_14313_amd import native
    say("case unrank", d, q)
    total, co, le, nz = orc.enumerate_window(d, q)
    K = q - d
    c, l, n = native.unrank_device(d, q, 0, total, max_nnz=max(1, K))
    c, l, n = c.cpu().numpy(), l.cpu().numpy(), n.cpu().numpy()
    assert np.array_equal(n, nz)
    for r in range(total):
        k = nz[r]
        assert np.array_equal(c[r, :k], co[r, :k]) and np.array_equal(l[r, :k], le[r, :k])


def test_unrank_device_large_window(api):
    from paper_2210_14313_amd import native
    d, q = 1000, 1003
    n = native.counts(d, q, "cc")[0]
    say("case unrank large")
    r0 = n - 100000
    c, l, z = native.unrank_device(d, q, r0, 100000)
    c, l, z = c.cpu().numpy(), l.cpu().numpy(), z.cpu().numpy()
    for r in list(range(0, 100000, 997)) + [99999]:
        ref = native.unrank(d, q, r0 + r)
        assert [(int(c[r, k]), int(l[r, k])) for k in range(z[r])] == ref


# --------------------------------------------------------------- errors
def test_errors_are_reported_before_launch(api):
    import torch
    from paper_2210_14313_amd import native, workloads as W
    bad = W.single(5, 5 + native.MAX_K + 1, "cc", "exp_sum", np.zeros(5))
    with pytest.raises(native.SgError) as e:
        native.Plan(bad.problems, "fp64")
    assert e.value.status == 2
    with pytest.raises(native.SgError) as e:
        native.Plan([], "fp64")
    assert e.value.status == 1
    bad = W.single(5, 4, "cc", "exp_sum", np.zeros(5))
    with pytest.raises(native.SgError) as e:
        native.Plan(bad.problems, "fp64")
    assert e.value.status == 1
    ok = W.single(3, 5, "cc", "exp_sum", np.zeros(3))
    plan = native.Plan(ok.problems, "fp64")
    assert native.lib().sg_plan_execute(plan.handle, None, None, None, None) == 1
    with pytest.raises(native.SgError) as e:
        native.unrank_device(3, 5, 5, 100)
    assert e.value.status == 1
    plan.close()


def test_set_schedule_validation_and_equivalence(api, orc):
    import torch
    from paper_2210_14313_amd import native, workloads as W
    b = W.random_small(12, 40, d_range=(1, 400), k_range=(0, 6))
    params = api.params_tensor(b)
    say("case set_schedule")
    plan = native.Plan(b.problems, "fp64")
    for bad in ((0, 4, 0, 0, 0), (65, 4, 0, 0, 0), (2, 3, 0, 0, 0), (2, 4, 2, 0, 0), (2, 4, 0, 2, 0), (2, 4, 0, 0, 2)):
        with pytest.raises(native.SgError) as e:
            plan.set_schedule(bad[0], bad[1], graph=bad[2], persistent=bad[3], cost_scaled=bad[4])
        assert e.value.status == 1
    ref = _fact_ref(orc, b)
    for cpl, gm, pq, cs in ((1, 1, 0, 0), (2, 4, 0, 1), (5, 2, 0, 0), (64, 1, 0, 1), (1, 4, 1, 0), (3, 2, 1, 1),
                            (64, 4, 1, 0)):
        plan.set_schedule(cpl, gm, persistent=bool(pq), cost_scaled=bool(cs))
        assert plan.info()["persistent"] == pq and plan.info()["cost_scaled"] == cs
        for rep in range(3):   # the work queue must come back reset after every launch
            got = plan.execute(params).cpu().numpy()
            assert np.max(np.abs(got - ref) / _scale(b, ref)) <= 1e-12, (cpl, gm, pq, rep)
    plan.close()


def test_persistent_queue_in_graph_replays(api, orc):
    import torch
    from paper_2210_14313_amd import native, workloads as W
    b = W.batched_uneven(n=512)
    params = api.params_tensor(b)
    ref = _fact_ref(orc, b)
    say("case persistent queue graph replays")
    for prec, tol in (("fp64", 1e-12), ("fp32e", 1e-7)):
        plan = native.Plan(b.problems, prec)
        plan.set_schedule(2, 4, graph=True, persistent=True)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        out = torch.empty(len(b), dtype=torch.float64, device="cuda")
        eager = plan.execute(params).clone()   # default stream: direct launch of the queue kernel
        for rep in range(4):                   # capture, then replays with host work between them
            out.fill_(float("nan"))
            s.wait_stream(torch.cuda.current_stream())
            plan.execute(params, out, stream=s)
            s.synchronize()
            assert torch.equal(out, eager), (prec, rep)
            got = out.cpu().numpy()
            assert np.max(np.abs(got - ref) / _scale(b, ref)) <= tol, (prec, rep)
        plan.close()


def test_persistent_queue_pops_and_resets(api, orc):
    """The persistent kernel with more descriptors than resident workgroups
    (one coordinate per lane on the 4096 batch): workgroups pop descriptors
    from the queue, and the last pop of a launch returns the counter to zero,
    so back-to-back launches and graph replays each run every descriptor;
    bitwise equal to the hardware-dispatch launch of the same descriptors."""
    import torch
    from paper_2210_14313_amd import native, workloads as W
    b = W.batched_uneven()
    params = api.params_tensor(b)
    say("case persistent queue pops")
    direct = native.Plan(b.problems, "fp64")
    direct.set_schedule(1, 4)
    nfwg = direct.info()["grid_blocks"]
    want = direct.execute(params).clone()
    direct.close()
    ref = _fact_ref(orc, b)
    assert np.max(np.abs(want.cpu().numpy() - ref) / _scale(b, ref)) <= 1e-12
    for graph in (False, True):
        plan = native.Plan(b.problems, "fp64")
        plan.set_schedule(1, 4, persistent=True, graph=graph)
        assert plan.info()["grid_blocks"] < nfwg           # the queue is popped
        s = torch.cuda.Stream()
        out = torch.empty(len(b), dtype=torch.float64, device="cuda")
        for rep in range(4):
            out.fill_(float("nan"))
            s.wait_stream(torch.cuda.current_stream())
            plan.execute(params, out, stream=s)
            plan.execute(params, out, stream=s)            # back to back on the stream
            s.synchronize()
            assert torch.equal(out, want), (graph, rep)
        plan.close()


def test_balanced_schedule(api, orc):
    """The balanced schedule (equal-cost waves, workgroups placed for equal
    per-CU load) on mixed batches: every result against the oracle and
    within its bound, for 1..4 waves per SIMD, in graph replays, on the
    4096 batch in every precision mode, and its rejections."""
    import torch
    from paper_2210_14313_amd import native, workloads as W
    b = W.random_small(13, 60, d_range=(1, 600), k_range=(0, 8), rules=W.ALL_RULES,
                       families=("exp_sum", "oscillatory", "product_peak", "gaussian"))
    params = api.params_tensor(b)
    ref = _fact_ref(orc, b)
    say("case balanced schedule small")
    plan = native.Plan(b.problems, "fp64")
    for bad in ((0, 0), (9, 0), (2, 2)):
        with pytest.raises(native.SgError) as e:
            plan.set_balanced(bad[0], graph=bool(bad[1]) if bad[1] < 2 else 2)
        assert e.value.status == 1
    for m in (1, 2, 3, 4):
        plan.set_balanced(m)
        inf = plan.info()
        assert inf["balanced"] == m and inf["persistent"] == 0
        out = torch.empty(len(b), dtype=torch.float64, device="cuda")
        bnd = torch.empty_like(out)
        plan.execute(params, out, bnd)
        got, bd = out.cpu().numpy(), bnd.cpu().numpy()
        assert np.max(np.abs(got - ref) / _scale(b, ref)) <= 1e-12, m
        assert np.all(np.abs(got - ref) <= bd), m
    plan.close()
    big = W.batched_uneven()
    bparams = api.params_tensor(big)
    bref = _fact_ref(orc, big)
    bscale = _scale(big, bref)
    s = torch.cuda.Stream()
    for prec, tol in (("fp64", 1e-12), ("fp32c", 1e-7), ("fp32e", 1e-7)):
        say("case balanced schedule batched_uneven", prec)
        plan = native.Plan(big.problems, prec)
        plan.set_balanced(2, graph=True)
        eager = plan.execute(bparams).clone()
        out = torch.empty(len(big), dtype=torch.float64, device="cuda")
        bnd = torch.empty_like(out)
        for rep in range(3):
            out.fill_(float("nan"))
            s.wait_stream(torch.cuda.current_stream())
            plan.execute(bparams, out, bnd, stream=s)
            s.synchronize()
            assert torch.equal(out, eager), (prec, rep)
        got, bd = out.cpu().numpy(), bnd.cpu().numpy()
        assert np.max(np.abs(got - bref) / bscale) <= tol, prec
        assert np.all(np.abs(got - bref) <= bd), prec
        plan.close()


def test_autotune_records_saved_and_loaded(api, orc, tmp_path):
    """Autotune on the device, save the records, load them into a new
    context: a plan of the same shape starts from the tuned schedule and
    still matches the oracle; the file names this device."""
    import torch
    from paper_2210_14313_amd import native, workloads as W
    b = W.random_small(21, 48, d_range=(1, 300), k_range=(0, 6))
    params = api.params_tensor(b)
    ref = _fact_ref(orc, b)
    say("case autotune records")
    ctx = native.Context()
    plan = native.Plan(b.problems, "fp64", ctx=ctx)
    out = torch.empty(len(b), dtype=torch.float64, device="cuda")
    plan.autotune(params, out)
    tuned = {k: v for k, v in plan.info().items() if k in ("coords_per_lane", "max_group", "persistent",
                                                         "cost_scaled", "balanced")}
    plan.close()
    path = str(tmp_path / "tune.json")
    ctx.save_tuning(path)
    doc = json.load(open(path))
    props = torch.cuda.get_device_properties(0)
    assert doc["compute_units"] == props.multi_processor_count
    assert doc["arch"].split(":")[0] == props.gcnArchName.split(":")[0]
    assert doc["version"] == native.version() and len(doc["entries"]) == 1
    ctx.close()
    ctx2 = native.Context()
    assert ctx2.load_tuning(path) == 1
    plan = native.Plan(b.problems, "fp64", ctx=ctx2)
    got_sched = {k: v for k, v in plan.info().items() if k in tuned}
    assert got_sched == tuned
    got = plan.execute(params).cpu().numpy()
    assert np.max(np.abs(got - ref) / _scale(b, ref)) <= 1e-12
    plan.close()
    ctx2.close()


@pytest.mark.parametrize("family", ["exp_sum", "oscillatory", "product_peak", "gaussian", "oscillatory_quadratic",
                                    "oscillatory_quadratic_linear"])
def test_plan_free_path_split_over_workgroups(api, orc, family):
    """sg_integrate sweeps an integrand on one workgroup up to d = 2048 (512
    for the complex sweep) and above splits it over ceil(d / 256) workgroups
    (at most 1024), joining their partials in a fixed order: FP64 against
    the oracle at sizes around the workgroup and split boundaries and beyond
    the cap, the same value on repeated calls, and graph replays of the
    split launch (the arrival counter must come back to zero after every
    launch)."""
    import torch
    from paper_2210_14313_amd import native, workloads as W
    rng = np.random.default_rng(31 + len(family))
    sizes = [(1, 4, "gl"), (255, 3, "cc"), (256, 2, "gp"), (257, 5, "gl"), (512, 2, "cc"), (513, 3, "gl"),
             (1000, 3, "tr"), (2048, 2, "gl"), (2049, 2, "cc")]
    if family != "product_peak":
        sizes += [(5000, 2, "cc"), (300000, 1, "cc")]
    for d, K, rule in sizes:
        prm = W.draw_params(rng, family, d)
        if family in ("exp_sum", "gaussian"):
            prm = prm * min(1.0, 30.0 / d)
        if family == "product_peak" and d > 1000:
            # factors 1 / (1 + (x - u)^2) near 1 keep the product in range
            prm = np.concatenate([np.ones(d), rng.uniform(0.4, 0.6, d)])
        b = W.single(d, d + K, rule, family, prm)
        p = b.problems[0]
        pr = torch.as_tensor(prm, dtype=torch.float64).cuda()
        say("case plan-free split", family, d, K, rule)
        out = torch.empty(1, dtype=torch.float64, device="cuda")
        bnd = torch.empty_like(out)
        native.integrate_one(p, pr, "fp64", out=out, bound=bnd)
        v1, b1 = out.item(), bnd.item()
        native.integrate_one(p, pr, "fp64", out=out, bound=bnd)
        assert (out.item(), bnd.item()) == (v1, b1)
        ref = orc.smolyak_factorised(p.d, p.q, p.rule, p.family, prm)
        scale = orc.accuracy_scale_one(p.d, p.q, p.rule, p.family, prm, ref)
        assert abs(v1 - ref) <= b1, (d, v1, ref, b1)
        assert abs(v1 - ref) <= 1e-12 * scale, (d, v1, ref)
    # graph replays of a split launch on a non-default stream
    d = 3000
    prm = W.draw_params(rng, family, d)
    if family in ("exp_sum", "gaussian"):
        prm = prm / d
    if family == "product_peak":
        prm = np.concatenate([np.ones(d), rng.uniform(0.4, 0.6, d)])
    p = W.single(d, d + 3, "cc", family, prm).problems[0]
    pr = torch.as_tensor(prm, dtype=torch.float64).cuda()
    eager = torch.empty(1, dtype=torch.float64, device="cuda")
    native.integrate_one(p, pr, "fp64", out=eager)
    s = torch.cuda.Stream()
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.cuda.CUDAGraph()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=s):
        native.integrate_one(p, pr, "fp64", out=out, stream=torch.cuda.current_stream())
    for rep in range(4):
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert out.item() == eager.item(), (family, rep)
        native.integrate_one(p, pr, "fp64", out=eager)      # eager work between replays
        torch.cuda.synchronize()
