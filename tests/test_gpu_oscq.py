"""GPU parity of the oscillatory-quadratic sweep cos(2 pi w + sum a_i (x_i - u_i)^2)
(the factorised sum with complex surpluses and complex truncated products:
sg_integrate, and plans, which give each such integrand a workgroup of the
complex kernel beside the forward sweep of the others), in every precision
mode (FP64; FP32 node values with compensated FP32 or FP64 within-rule
sums, FP64 products), against the oracle's point-by-point sum (small d) and
its binary128 factorised sum (any d), with the stated bound; the sine of
Test 1 ((4.1), on [-1,1]^2 mapped to the unit cube); the block variant; the
complex reverse sweep against the oracle's gradient.

Tolerance: within the stated bound, and within 1e-12 (FP64) or 1e-6 (FP32
modes) relative to the oracle's accuracy scale (the modulus of the complex
Smolyak sum, sqrt(Q(w)^2 + Q(w - 1/4)^2)).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FAM = "oscillatory_quadratic"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2210_14313_amd import native
    native.lib()
    return torch


def _one(problem, prm, precision="fp64"):
    import torch
    from paper_2210_14313_amd import native
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    bound = torch.empty(1, dtype=torch.float64, device="cuda")
    native.integrate_one(problem, torch.as_tensor(prm, dtype=torch.float64).cuda(), precision, out=out, bound=bound)
    torch.cuda.synchronize()
    return out.item(), bound.item()


def native_info(batch, precision):
    from paper_2210_14313_amd import native
    plan = native.Plan(batch.problems, precision)
    try:
        return plan.info()
    finally:
        plan.close()


def _mod(batch, ref):
    import oracle
    return oracle.accuracy_scale(batch, np.atleast_1d(ref))


TOL = {"fp64": 1e-12, "fp32c": 1e-6, "fp32e": 1e-6}
MODES = ["fp64", "fp32c", "fp32e"]


def _check(got, bnd, ref, scale, extra=0.0, precision="fp64"):
    assert abs(got - ref) <= bnd + extra, (got, ref, bnd)
    assert abs(got - ref) <= TOL[precision] * scale, (got, ref, abs(got - ref) / scale)


@pytest.mark.parametrize("precision", MODES)
@pytest.mark.parametrize("seed", [1, 2])
def test_oscq_small_random_vs_point_oracle(torch_dev, orc, seed, precision):
    from paper_2210_14313_amd import workloads as W
    b = W.random_small(900 + seed, 40, d_range=(1, 10), k_range=(0, 6), families=(FAM,), rules=W.ALL_RULES)
    say("case oscq small", seed, precision)
    for i, p in enumerate(b.problems):
        r = orc.smolyak_points(p.d, p.q, p.rule, p.family, b.param_slice(i))
        got, bnd = _one(p, b.param_slice(i), precision)
        # the point oracle's own rounding (extended precision) is below
        # 8 * 2^-64 * (A + |f(c)|)
        _check(got, bnd, r["q"], _mod(b.subset([i]), r["q"])[0], 8 * 2.0 ** -64 * (r["A"] + abs(r["fc"])),
               precision)


@pytest.mark.parametrize("d,K,rule,scale", [(1, 8, "gp", 1.0), (3, 5, "cc", 5.0), (64, 4, "tr", 1.0),
                                            (255, 3, "gl_paper", 1.0), (257, 6, "gl", 1.0), (300, 8, "cc", 0.5),
                                            (1000, 2, "cc", 1.0), (1000, 4, "gp", 1.0)])
@pytest.mark.parametrize("precision", MODES)
def test_oscq_edges_vs_factorised_oracle(torch_dev, orc, d, K, rule, scale, precision):
    from paper_2210_14313_amd import workloads as W
    rng = np.random.default_rng(d + 100 * K)
    prm = W.draw_params(rng, FAM, d)
    prm[1:1 + d] *= scale
    b = W.single(d, d + K, rule, FAM, prm)
    say("case oscq edge", d, K, rule, scale, precision)
    ref = orc.batch_factorised(b)[0]
    got, bnd = _one(b.problems[0], prm, precision)
    _check(got, bnd, ref, _mod(b, ref)[0], precision=precision)


def test_oscq_paper_test_1_sine(torch_dev, orc):
    # sin(2 pi + 10 x_1^2 + 5 x_2^2) on [-1,1]^2: x = 2t - 1 gives
    # 10 x^2 = 40 (t - 1/2)^2, and sin(theta) = cos(theta - pi/2), so
    # w = 3/4, a = (40, 20), u = (1/2, 1/2); the mean over the unit cube
    from paper_2210_14313_amd import workloads as W
    prm = np.array([0.75, 40.0, 20.0, 0.5, 0.5])
    for q in range(3, 11):
        b = W.single(2, q, "gp", FAM, prm)
        say("case oscq test 1", q)
        r = orc.smolyak_points(2, q, "gp", FAM, prm)
        got, bnd = _one(b.problems[0], prm)
        _check(got, bnd, r["q"], _mod(b, r["q"])[0], 8 * 2.0 ** -64 * (r["A"] + abs(r["fc"])))


def test_oscq_deterministic_in_every_mode(torch_dev, orc):
    # the split launch (d = 500: two workgroups joined in order) repeats
    # bitwise in each mode; the FP32 modes compute their own node values
    from paper_2210_14313_amd import workloads as W
    rng = np.random.default_rng(5)
    prm = W.draw_params(rng, FAM, 500)
    prm[1:501] *= 50.0                      # sizeable surpluses
    b = W.single(500, 505, "cc", FAM, prm)
    ref = orc.batch_factorised(b)[0]
    vals = {}
    for prec in MODES:
        v1, b1 = _one(b.problems[0], prm, prec)
        v2, b2 = _one(b.problems[0], prm, prec)
        assert v1 == v2 and b1 == b2, prec
        _check(v1, b1, ref, _mod(b, ref)[0], precision=prec)
        vals[prec] = v1
    assert vals["fp32c"] != vals["fp64"] and vals["fp32e"] != vals["fp64"]


@pytest.mark.parametrize("precision", MODES)
def test_oscq_in_mixed_plans(torch_dev, orc, precision):
    # plans compute the family on the complex sweep in their precision mode
    from paper_2210_14313_amd import api, workloads as W
    b = W.concat([W.random_small(950, 30, d_range=(1, 300), k_range=(0, 6), families=(FAM,), rules=W.ALL_RULES),
                  W.random_small(951, 40, d_range=(1, 120), k_range=(0, 6)),
                  W.random_small(952, 10, d_range=(1, 60), k_range=(0, 5), families=("gaussian",))])
    say("case oscq mixed plan", precision)
    ref = orc.batch_factorised(b)
    vals, bnd = api.integrate(b, precision, with_bound=True)
    got, bnd = vals.cpu().numpy(), bnd.cpu().numpy()
    assert np.all(np.abs(got - ref) <= bnd), np.max(np.abs(got - ref) / bnd)
    fam = np.array([p.family for p in b.problems])
    sel = fam == FAM
    err = np.max(np.abs(got[sel] - ref[sel]) / _mod(b, ref)[sel])
    say("  max error / accuracy scale", err)
    assert err <= TOL[precision]
    info = native_info(b, precision)
    assert info["fp64_complex"] == int(np.sum(sel))
    for i in np.flatnonzero(sel)[:5]:                      # the same value as the one-shot path
        one = b.subset([int(i)])
        if one.problems[0].d > 256:
            continue                                       # split launch: another join order
        v, _ = _one(one.problems[0], one.param_slice(0), precision)
        assert v == got[i]


def test_oscq_only_plan_autotuned_on_a_stream(torch_dev, orc):
    import torch
    from paper_2210_14313_amd import api, native, workloads as W
    b = W.concat([W.random_small(960, 12, d_range=(200, 1000), k_range=(1, 5), families=(FAM,)),
                  W.oscillatory_quadratic_d1000()])
    say("case oscq-only plan")
    ref = orc.batch_factorised(b)
    params = api.params_tensor(b)
    plan = native.Plan(b.problems, "fp64")
    s = torch.cuda.Stream()
    try:
        out = torch.empty(len(b), dtype=torch.float64, device="cuda")
        bound = torch.empty_like(out)
        plan.autotune(params, out, stream=s)
        runs = []
        for _ in range(3):
            plan.execute(params, out, bound, stream=s)
            s.synchronize()
            runs.append(out.cpu().numpy().copy())
        bnd = bound.cpu().numpy()
    finally:
        plan.close()
    for r in runs[1:]:
        assert np.array_equal(r, runs[0])
    assert np.all(np.abs(runs[0] - ref) <= bnd)
    assert np.max(np.abs(runs[0] - ref) / _mod(b, ref)) <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_oscq_block_variant(torch_dev, orc, precision):
    # blocks of 5 coordinates, each block's complex value from two
    # sub-problems (w = 0 and w = -1/4) of the complex sweep, against the
    # oracle's block rule; mixed with the linear oscillatory family
    from oracle import blocked as OB
    from paper_2210_14313_amd import api, workloads as W
    b = W.concat([W.random_small(970, 12, d_range=(3, 40), k_range=(1, 5), families=(FAM,), rules=W.ALL_RULES),
                  W.random_small(971, 8, d_range=(3, 40), k_range=(1, 5), families=("oscillatory",))])
    say("case oscq blocked", precision)
    ref = np.array([OB.smolyak_blocked(p.d, p.q, p.rule, p.family, b.param_slice(i), 5)
                    for i, p in enumerate(b.problems)])
    vals, bnd = api.integrate(b, precision, with_bound=True, block_dims=5)
    got, bnd = vals.cpu().numpy(), bnd.cpu().numpy()
    assert np.all(np.abs(got - ref) <= bnd), np.max(np.abs(got - ref) / bnd)
    fam = np.array([p.family for p in b.problems])
    sel = fam == FAM
    assert np.max(np.abs(got[sel] - ref[sel]) / _mod(b, ref)[sel]) <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_oscq_reverse_sweep_vs_oracle_gradient(torch_dev, orc, precision):
    """The complex reverse sweep (FP64 in every mode) against the oracle's
    binary128 factorised gradient (dQ/dw, dQ/da_t, dQ/du_t), in a plan that
    mixes it with the real families, including integrands whose threads hold
    several coordinates (d > 256, the workspace path), with a non-trivial
    grad_out."""
    import torch
    from paper_2210_14313_amd import api, native, workloads as W
    rng = np.random.default_rng(41)
    b = W._Builder("oscq_grad_mix")
    shapes = [(1, 0, "cc"), (3, 2, "gl"), (20, 4, "cc"), (64, 3, "gp"), (255, 2, "tr"), (256, 5, "gl"),
              (257, 3, "cc"), (600, 4, "gl"), (1000, 2, "gp")]
    for d, K, rule in shapes:
        b.add(d, d + K, rule, FAM, W.draw_params(rng, FAM, d))
    for d, K, rule, fam in [(40, 3, "cc", "oscillatory"), (70, 4, "gl", "exp_sum"), (33, 2, "gp", "gaussian")]:
        b.add(d, d + K, rule, fam, W.draw_params(rng, fam, d))
    b = b.build()
    say("case oscq reverse sweep", precision)
    params = api.params_tensor(b)
    gout = torch.tensor(rng.uniform(0.5, 2.0, len(b)), dtype=torch.float64, device="cuda")
    plan = native.Plan(b.problems, precision)
    try:
        got = plan.execute_grad(params, gout).cpu().numpy()
    finally:
        plan.close()
    gw = gout.cpu().numpy()
    for i, p in enumerate(b.problems):
        ref = gw[i] * orc.smolyak_factorised_grad(p.d, p.q, p.rule, p.family, b.param_slice(i))
        sl = slice(p.param_offset, p.param_offset + len(ref))
        scale = max(np.max(np.abs(ref)), 1e-300)
        err = np.max(np.abs(got[sl] - ref)) / scale
        tol = 1e-12 if (p.family == FAM or precision == "fp64") else 1e-6
        assert err <= tol, (i, p.d, p.q, p.rule, p.family, err)


@pytest.mark.parametrize("persistent", [False, True])
def test_oscq_plan_graph_replays(torch_dev, orc, persistent):
    # a plan holding the family, its launches captured into a graph (on a
    # non-default stream) and replayed with eager work and host
    # synchronisation between the replays; every replay equals the eager
    # (direct-launch) result bitwise
    import torch
    from paper_2210_14313_amd import api, native, workloads as W
    b = W.concat([W.random_small(980, 10, d_range=(1, 400), k_range=(0, 6), families=(FAM,)),
                  W.random_small(981, 30, d_range=(1, 200), k_range=(0, 6))])
    say("case oscq graph replays", persistent)
    params = api.params_tensor(b)
    ref = orc.batch_factorised(b)
    plan = native.Plan(b.problems, "fp64")
    try:
        plan.set_schedule(2, 4, graph=True, persistent=persistent)
        eager = plan.execute(params).clone()           # default stream: direct launches
        assert np.max(np.abs(eager.cpu().numpy() - ref) / _mod(b, ref)) <= 1e-12
        s = torch.cuda.Stream()
        out = torch.empty(len(b), dtype=torch.float64, device="cuda")
        for _ in range(4):                             # capture, then replays
            out.fill_(float("nan"))
            torch.cuda.synchronize()
            s.wait_stream(torch.cuda.current_stream())
            plan.execute(params, out, stream=s)
            s.synchronize()
            assert torch.equal(out, eager)
            torch.cuda.synchronize()
    finally:
        plan.close()


def test_oscq_degenerate_and_large_coefficients(torch_dev, orc):
    # K = 0 (the midpoint rule: cos(2 pi w + sum a (1/2 - u)^2)), d = 1, and
    # quadratic coefficients a ~ 1e3 (arguments of the sines in the
    # hundreds): one-shot and in a plan, within the bound
    from paper_2210_14313_amd import api, workloads as W
    rng = np.random.default_rng(77)
    cases = []
    for d, K, scale in [(1, 0, 1.0), (5, 0, 1.0), (1, 8, 1.0), (1, 8, 300.0), (2, 6, 1000.0), (7, 3, 200.0)]:
        prm = W.draw_params(rng, FAM, d)
        prm[1:1 + d] *= scale
        cases.append(W.single(d, d + K, "cc" if K % 2 else "gl", FAM, prm))
    b = W.concat(cases)
    say("case oscq degenerate / large")
    ref = orc.batch_factorised(b)
    mod = _mod(b, ref)
    for i, p in enumerate(b.problems):
        pt = orc.smolyak_points(p.d, p.q, p.rule, p.family, b.param_slice(i))
        assert abs(pt["q"] - ref[i]) <= 1e-12 * mod[i] + 8 * 2.0 ** -64 * (pt["A"] + abs(pt["fc"]))
        for prec in MODES:
            v, bd = _one(p, b.param_slice(i), prec)
            assert abs(v - ref[i]) <= bd, (i, prec, v, ref[i], bd)
            if p.q == p.d:
                w, a, u = b.param_slice(i)[0], b.param_slice(i)[1:1 + p.d], b.param_slice(i)[1 + p.d:]
                assert abs(v - np.cos(2 * np.pi * w + np.sum(a * (0.5 - u) ** 2))) <= 1e-14
    for prec in MODES:
        vals, bnd = api.integrate(b, prec, with_bound=True)
        got, bnd = vals.cpu().numpy(), bnd.cpu().numpy()
        assert np.all(np.abs(got - ref) <= bnd), prec


# ------------------------------------------ with a linear term in the phase
FAML = "oscillatory_quadratic_linear"


@pytest.mark.parametrize("precision", MODES)
@pytest.mark.parametrize("seed", [3, 4])
def test_oscql_small_random_vs_point_oracle(torch_dev, orc, seed, precision):
    from paper_2210_14313_amd import workloads as W
    b = W.random_small(900 + seed, 30, d_range=(1, 10), k_range=(0, 6), families=(FAML,), rules=W.ALL_RULES)
    say("case oscql small", seed, precision)
    for i, p in enumerate(b.problems):
        r = orc.smolyak_points(p.d, p.q, p.rule, p.family, b.param_slice(i))
        got, bnd = _one(p, b.param_slice(i), precision)
        _check(got, bnd, r["q"], _mod(b.subset([i]), r["q"])[0], 8 * 2.0 ** -64 * (r["A"] + abs(r["fc"])),
               precision)


@pytest.mark.parametrize("d,K,rule,lin_only", [(1, 8, "gp", False), (3, 5, "cc", True), (64, 4, "tr", False),
                                               (257, 6, "gl", False), (600, 3, "cc", True), (1000, 4, "gp", False)])
@pytest.mark.parametrize("precision", MODES)
def test_oscql_edges_vs_factorised_oracle(torch_dev, orc, d, K, rule, lin_only, precision):
    # lin_only: every other coordinate purely linear (a = 0), the rest purely
    # quadratic (c = 0), as in (4.2)
    from paper_2210_14313_amd import workloads as W
    rng = np.random.default_rng(d + 100 * K + 7)
    prm = W.draw_params(rng, FAML, d)
    if lin_only:
        prm[1:1 + d:2] = 0.0
        prm[1 + 2 * d + 1::2] = 0.0
    b = W.single(d, d + K, rule, FAML, prm)
    say("case oscql edge", d, K, rule, lin_only, precision)
    ref = orc.batch_factorised(b)[0]
    got, bnd = _one(b.problems[0], prm, precision)
    _check(got, bnd, ref, _mod(b, ref)[0], precision=precision)


def _test_2_sine_params():
    # sin(2 pi + 10 x1^2 + 5 x2^2 + 5 x3) on [-1,1]^3: x = 2t - 1 gives
    # 10 x1^2 = 40 (t1 - 1/2)^2, 5 x2^2 = 20 (t2 - 1/2)^2, 5 x3 = 10 t3 - 5,
    # and sin(theta) = cos(theta - pi/2): w = 3/4 - 5 / (2 pi) (mod 1),
    # a = (40, 20, 0), u = 1/2, c = (0, 0, 10); the mean over the unit cube
    w = (0.75 - 5.0 / (2.0 * np.pi)) % 1.0
    return np.array([w, 40.0, 20.0, 0.0, 0.5, 0.5, 0.5, 0.0, 0.0, 10.0])


def test_oscql_paper_test_2_sine(torch_dev, orc):
    import torch
    from paper_2210_14313_amd import native, workloads as W
    prm = _test_2_sine_params()
    for K in range(0, 9):
        b = W.single(3, 3 + K, "gp", FAML, prm)
        say("case oscql test 2", K)
        r = orc.smolyak_points(3, 3 + K, "gp", FAML, prm)
        for prec in MODES:
            got, bnd = _one(b.problems[0], prm, prec)
            _check(got, bnd, r["q"], _mod(b, r["q"])[0], 8 * 2.0 ** -64 * (r["A"] + abs(r["fc"])), prec)
        pv = native.integrate_points(b.problems[0], torch.as_tensor(prm).cuda()).item()
        assert abs(pv - r["q"]) <= 1e-12 * _mod(b, r["q"])[0], (K, pv, r["q"])


@pytest.mark.parametrize("precision", MODES)
def test_oscql_in_mixed_plans_with_gradient(torch_dev, orc, precision):
    # both complex families beside the real ones in one plan: values, the
    # family count in the plan info, and the reverse sweep against the
    # oracle's gradient (dw, da, du, dc)
    import torch
    from paper_2210_14313_amd import api, native, workloads as W
    b = W.concat([W.random_small(990, 20, d_range=(1, 400), k_range=(0, 6), families=(FAML,), rules=W.ALL_RULES),
                  W.random_small(991, 10, d_range=(1, 300), k_range=(0, 6), families=(FAM,)),
                  W.random_small(992, 20, d_range=(1, 120), k_range=(0, 6))])
    say("case oscql mixed plan", precision)
    ref = orc.batch_factorised(b)
    vals, bnd = api.integrate(b, precision, with_bound=True)
    got, bnd = vals.cpu().numpy(), bnd.cpu().numpy()
    assert np.all(np.abs(got - ref) <= bnd), np.max(np.abs(got - ref) / bnd)
    fam = np.array([p.family for p in b.problems])
    sel = (fam == FAML) | (fam == FAM)
    err = np.max(np.abs(got[sel] - ref[sel]) / _mod(b, ref)[sel])
    say("  max error / accuracy scale", err)
    assert err <= TOL[precision]
    assert native_info(b, precision)["fp64_complex"] == int(np.sum(sel))
    params = api.params_tensor(b)
    rng = np.random.default_rng(993)
    gout = torch.tensor(rng.uniform(0.5, 2.0, len(b)), dtype=torch.float64, device="cuda")
    plan = native.Plan(b.problems, precision)
    try:
        g = plan.execute_grad(params, gout).cpu().numpy()
    finally:
        plan.close()
    gw = gout.cpu().numpy()
    for i, p in enumerate(b.problems):
        if p.family != FAML:
            continue
        gr = gw[i] * orc.smolyak_factorised_grad(p.d, p.q, p.rule, p.family, b.param_slice(i))
        sl = slice(p.param_offset, p.param_offset + len(gr))
        e = np.max(np.abs(g[sl] - gr)) / max(np.max(np.abs(gr)), 1e-300)
        assert e <= 1e-12, (i, p.d, p.q, p.rule, e)


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_oscql_block_variant(torch_dev, orc, precision):
    from oracle import blocked as OB
    from paper_2210_14313_amd import api, workloads as W
    b = W.random_small(995, 12, d_range=(3, 40), k_range=(1, 5), families=(FAML,), rules=W.ALL_RULES)
    say("case oscql blocked", precision)
    ref = np.array([OB.smolyak_blocked(p.d, p.q, p.rule, p.family, b.param_slice(i), 5)
                    for i, p in enumerate(b.problems)])
    vals, bnd = api.integrate(b, precision, with_bound=True, block_dims=5)
    got, bnd = vals.cpu().numpy(), bnd.cpu().numpy()
    assert np.all(np.abs(got - ref) <= bnd), np.max(np.abs(got - ref) / bnd)
    assert np.max(np.abs(got - ref) / _mod(b, ref)) <= TOL[precision]


def test_box_map_paper_domains_on_the_gpu(torch_dev, orc):
    """api.integrate_one with box=(-1, 1): (4.2)'s sine on [-1,1]^3 (eight
    times the unit-cube value of the mapped integrand, against the oracle),
    and (4.1)'s exp(5 x1^2 + 5 x2^2) on [-1,1]^2 (four times the unit-cube
    gaussian c = 20, u = 1/2, bitwise)."""
    import torch
    from paper_2210_14313_amd import api, native, workloads as W
    p = np.array([0.75, 10.0, 5.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 5.0])   # sin(theta) = cos(theta - pi/2)
    for K in (2, 5, 8):
        v, bnd = api.integrate_one(FAML, p, 3, 3 + K, "gp", box=(-1.0, 1.0), with_bound=True)
        up = _test_2_sine_params()
        ref = 8.0 * orc.smolyak_factorised(3, 3 + K, "gp", FAML, up)
        scale = 8.0 * _mod(W.single(3, 3 + K, "gp", FAML, up), ref / 8.0)[0]
        assert abs(v - ref) <= 1e-12 * scale, (K, v, ref)
        assert abs(v - ref) <= bnd + 1e-14 * scale
    g = api.integrate_one("gaussian", [5.0, 5.0, 0.0, 0.0], 2, 7, "gp", box=(-1.0, 1.0))
    b = W.single(2, 7, "gp", "gaussian", np.array([20.0, 20.0, 0.5, 0.5]))
    u = native.integrate_one(b.problems[0], torch.as_tensor(b.params).cuda()).item()
    assert g == 4.0 * u
