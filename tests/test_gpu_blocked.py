"""GPU parity of the block (tensor-product) variant (sg_plan_create_blocked)
against the oracle's block rule, through the C ABI.

Tolerances as for the plain rule: FP64 within 1e-12 relative (oscillatory:
relative to the modulus of the complex block rule) and within the stated bound; the FP32 modes within
the stated bound, which the combine step propagates from the blocks' bounds.
"""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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


def _scale(batch, ref, m):
    """|Q|, and for the oscillatory family the modulus of the complex block
    rule, sqrt(Q(w)^2 + Q(w - 1/4)^2) (the block rule is linear in the
    integrand, so Q(w - 1/4) is the imaginary part)."""
    import oracle
    from oracle import blocked as B
    sc = np.abs(ref).copy()
    for i, p in enumerate(batch.problems):
        if p.family in oracle.OSCILLATORY_FAMILIES:
            prm = np.array(batch.param_slice(i), copy=True)
            prm[0] -= 0.25
            sc[i] = np.hypot(ref[i], B.smolyak_blocked(p.d, p.q, p.rule, p.family, prm, m, "factorised"))
    return sc


def _blocked_ref(batch, m, method):
    from oracle import blocked as B
    return np.array([B.smolyak_blocked(p.d, p.q, p.rule, p.family, batch.param_slice(i), m, method)
                     for i, p in enumerate(batch.problems)])


def _run(batch, precision, m, autotune=False):
    import torch
    from paper_2210_14313_amd import api, native
    params = api.params_tensor(batch)
    plan = native.Plan(batch.problems, precision, block_dims=m)
    try:
        out = torch.empty(len(batch), dtype=torch.float64, device="cuda")
        bound = torch.empty_like(out)
        if autotune:
            plan.autotune(params, out, stream=torch.cuda.Stream())
        plan.execute(params, out, bound)
        torch.cuda.synchronize()
        return out.cpu().numpy(), bound.cpu().numpy(), plan.info()
    finally:
        plan.close()


@pytest.mark.parametrize("m", [1, 2, 3, 5])
@pytest.mark.parametrize("seed", [1, 2])
def test_small_random_blocked_fp64(torch_dev, orc, seed, m):
    from paper_2210_14313_amd import workloads as W
    b = W.random_small(100 + seed, 48, d_range=(1, 12), k_range=(0, 5))
    say("case blocked small fp64 seed", seed, "m", m)
    got, bnd, _ = _run(b, "fp64", m)
    ref = _blocked_ref(b, m, "points")
    err = np.abs(got - ref) / _scale(b, ref, m)
    assert np.max(err) <= 1e-12, (np.argmax(err), np.max(err))
    assert np.all(np.abs(got - ref) <= bnd + 1e-300)


@pytest.mark.parametrize("prec", ["fp32c", "fp32e"])
@pytest.mark.parametrize("m", [2, 4])
def test_small_random_blocked_fp32(torch_dev, orc, prec, m):
    from paper_2210_14313_amd import workloads as W
    b = W.random_small(200 + m, 48, d_range=(1, 12), k_range=(0, 5))
    say("case blocked small", prec, "m", m)
    got, bnd, _ = _run(b, prec, m)
    ref = _blocked_ref(b, m, "points")
    assert np.all(np.abs(got - ref) <= bnd), np.max(np.abs(got - ref) / bnd)


@pytest.mark.parametrize("family", ["exp_sum", "oscillatory", "product_peak"])
def test_one_block_matches_the_plain_plan(torch_dev, family):
    from paper_2210_14313_amd import api, workloads as W
    rng = np.random.default_rng(5)
    b = W.single(40, 44, "cc", family, W.draw_params(rng, family, 40))
    say("case blocked one block", family)
    plain, pb = api.integrate(b, "fp64", with_bound=True)
    plain, pb = plain.cpu().numpy(), pb.cpu().numpy()
    import oracle
    p = b.problems[0]
    sc = oracle.accuracy_scale_one(p.d, p.q, p.rule, p.family, b.param_slice(0),
                                   oracle.smolyak_factorised(p.d, p.q, p.rule, p.family, b.param_slice(0)))
    for m in (40, 64):
        got, bnd, _ = _run(b, "fp64", m)
        assert abs(got[0] - plain[0]) <= bnd[0] + pb[0]
        assert abs(got[0] - plain[0]) <= 1e-13 * sc


def test_high_dimension_paper_setting(torch_dev, orc):
    # d = 1000 in blocks of 10 (the step of Table 4.9), each block with its
    # own budget; against the oracle's block rule (binary128 blocks)
    from paper_2210_14313_amd import workloads as W
    rng = np.random.default_rng(1003)
    probs = []
    for fam, rule, K in (("exp_sum", "gl", 4), ("oscillatory", "cc", 3), ("product_peak", "gl_paper", 6)):
        d = 1000 if fam != "product_peak" else 997
        prm = W.draw_params(rng, fam, d)
        if fam == "exp_sum":
            prm = prm / d
        probs.append((d, d + K, rule, fam, prm))
    b = W.concat([W.single(*pr) for pr in probs])
    say("case blocked d1000 m10")
    ref = _blocked_ref(b, 10, "factorised")
    for prec in ("fp64", "fp32c"):
        got, bnd, info = _run(b, prec, 10)
        assert np.all(np.abs(got - ref) <= bnd), (prec, got, ref, bnd)
        if prec == "fp64":
            assert np.max(np.abs(got - ref) / _scale(b, ref, 10)) <= 1e-12
    assert info["effective_points"] == 2 ** 64 - 1     # the tensor product's count saturates


def test_blocked_autotuned_and_graph_replays(torch_dev, orc):
    import torch
    from paper_2210_14313_amd import api, native, workloads as W
    b = W.random_small(300, 96, d_range=(8, 40), k_range=(1, 4))
    say("case blocked autotune")
    ref = _blocked_ref(b, 6, "factorised")
    params = api.params_tensor(b)
    plan = native.Plan(b.problems, "fp32c", block_dims=6)
    s = torch.cuda.Stream()
    try:
        out = torch.empty(len(b), dtype=torch.float64, device="cuda")
        bound = torch.empty_like(out)
        plan.autotune(params, out, stream=s)
        first = None
        for rep in range(4):
            out.fill_(0.0)
            plan.execute(params, out, bound, stream=s)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            assert np.all(np.abs(got - ref) <= bound.cpu().numpy())
            if first is None:
                first = got.copy()
            assert np.array_equal(got, first)      # bitwise reproducible
        # one graph of the three launches (gather, forward, combine), replayed
        # with eager work and synchronisations in between
        for graph, persistent in ((True, True), (True, False), (False, True)):
            plan.set_schedule(3, 2, graph=graph, persistent=persistent)
            assert plan.info()["graph"] == int(graph)
            prev = None
            for rep in range(3):
                out.fill_(0.0)
                plan.execute(params, out, bound, stream=s)
                torch.cuda.synchronize()
                got = out.cpu().numpy()
                assert np.all(np.abs(got - ref) <= bound.cpu().numpy()), (graph, persistent, rep)
                if prev is not None:
                    assert np.array_equal(got, prev)
                prev = got.copy()
    finally:
        plan.close()


def test_blocked_rejections(torch_dev):
    from paper_2210_14313_amd import api, native, workloads as W
    L = native.lib()
    b = W.single(6, 9, "cc", "exp_sum", np.full(6, 0.3))
    arr = native.make_problems(b.problems)
    h = ctypes.c_void_p()
    ctx = native.default_context()
    assert L.sg_plan_create_blocked(ctx.handle, arr, 1, 0, 0, ctypes.byref(h)) == 1   # block_dims < 1
    assert not h.value
    corner = W.single(4, 6, "cc", "corner_peak", np.full(4, 0.25))
    with pytest.raises(native.SgError) as e:
        native.Plan(corner.problems, "fp64", block_dims=2)
    assert e.value.status == 2
    plan = native.Plan(b.problems, "fp64", block_dims=2)
    try:
        params = api.params_tensor(b)
        import torch
        with pytest.raises(native.SgError) as e:
            plan.execute_grad(params, torch.ones(1, dtype=torch.float64, device="cuda"))
        assert e.value.status == 2
    finally:
        plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32e"])
def test_oscillatory_blocks_with_large_phases(torch_dev, orc, prec):
    # oscillatory blocks are swept once with their centre phase cancelled
    # and rotated back in the combine: phases theta_b = sum a_t / 2 of up to
    # about 10 rad, coefficients beyond |a| = 2 (the sweep's table-driven
    # path), and a ragged last block (d = 23, 30 in blocks of 7)
    from paper_2210_14313_amd import workloads as W
    rng = np.random.default_rng(707)
    parts = []
    for d, rule in ((23, "cc"), (30, "gl"), (23, "tr"), (30, "gp")):
        prm = np.concatenate([[rng.uniform(0.0, 1.0)], rng.uniform(-3.0, 3.0, d)])
        parts.append(W.single(d, d + 3, rule, "oscillatory", prm))
    b = W.concat(parts)
    say("case blocked oscillatory large phases", prec)
    ref = _blocked_ref(b, 7, "factorised")
    got, bnd, _ = _run(b, prec, 7)
    assert np.all(np.abs(got - ref) <= bnd), np.abs(got - ref) / bnd
    if prec == "fp64":
        err = np.abs(got - ref) / _scale(b, ref, 7)
        assert np.max(err) <= 1e-12, err
