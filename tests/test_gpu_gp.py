"""GPU parity of the Gauss-Patterson rule (Example 3 of Section 2.2, level
map of Section 5.4) through every path: the batched forward sweep in the
three precision modes (compiled tables for K <= 6, table-driven K = 7, 8),
the reverse sweep, the point-by-point path and the block variant, against
the oracle's own Gauss-Patterson construction.

Tolerances as for the other rules: FP64 within 1e-12 relative (oscillatory:
to the oracle's accuracy scale: the modulus of the complex Smolyak sum) and
within the stated bound; FP32 modes within the bound.
"""
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


def _scale(batch, ref):
    import oracle
    return oracle.accuracy_scale(batch, ref)


def _run(batch, precision):
    from paper_2210_14313_amd import api
    vals, bnd = api.integrate(batch, precision, with_bound=True)
    return vals.cpu().numpy(), bnd.cpu().numpy()


@pytest.mark.parametrize("seed", [1, 2])
def test_gp_small_random_all_modes(torch_dev, orc, seed):
    from paper_2210_14313_amd import workloads as W
    b = W.random_small(500 + seed, 48, d_range=(1, 10), k_range=(0, 6), rules=("gp",))
    say("case gp small random", seed)
    ref = np.array([orc.smolyak_points(p.d, p.q, p.rule, p.family, b.param_slice(i))["q"]
                    for i, p in enumerate(b.problems)])
    got, bnd = _run(b, "fp64")
    assert np.max(np.abs(got - ref) / _scale(b, ref)) <= 1e-12
    assert np.all(np.abs(got - ref) <= bnd)
    for prec in ("fp32c", "fp32e"):
        got, bnd = _run(b, prec)
        assert np.all(np.abs(got - ref) <= bnd), prec


@pytest.mark.parametrize("d,K,family", [(1, 8, "exp_sum"), (3, 7, "oscillatory"), (20, 8, "product_peak"),
                                        (65, 7, "exp_sum"), (200, 6, "oscillatory"), (257, 3, "product_peak"),
                                        (1000, 4, "exp_sum")])
def test_gp_edges_and_table_driven_levels(torch_dev, orc, d, K, family):
    from paper_2210_14313_amd import workloads as W
    rng = np.random.default_rng(7000 + d + K)
    prm = W.draw_params(rng, family, d)
    if family == "exp_sum":
        prm = prm / max(1.0, d / 10.0)
    b = W.single(d, d + K, "gp", family, prm)
    say("case gp edge", d, K, family)
    ref = orc.batch_factorised(b)
    for prec in ("fp64", "fp32c", "fp32e"):
        got, bnd = _run(b, prec)
        assert abs(got[0] - ref[0]) <= bnd[0], (prec, got, ref, bnd)
        if prec == "fp64":
            assert abs(got[0] - ref[0]) <= 1e-12 * _scale(b, ref)[0]


def test_gp_gradient(torch_dev, orc):
    import torch
    from paper_2210_14313_amd import api, native, workloads as W
    b = W.random_small(77, 24, d_range=(1, 300), k_range=(0, 6), rules=("gp",))
    say("case gp gradient")
    params = api.params_tensor(b)
    plan = native.Plan(b.problems, "fp64")
    try:
        g = torch.zeros_like(params)
        plan.execute_grad(params, torch.ones(len(b), dtype=torch.float64, device="cuda"), g)
        torch.cuda.synchronize()
        g = g.cpu().numpy()
    finally:
        plan.close()
    for i, p in enumerate(b.problems):
        ref = orc.smolyak_factorised_grad(p.d, p.q, p.rule, p.family, b.param_slice(i))
        n = len(ref)
        sl = g[p.param_offset:p.param_offset + n]
        assert np.max(np.abs(sl - ref)) <= 1e-11 * max(np.max(np.abs(ref)), 1e-300), (i, p)


@pytest.mark.parametrize("d,K,family", [(4, 6, "oscillatory"), (12, 4, "product_peak"), (30, 3, "exp_sum"),
                                        (2, 8, "corner_peak")])
def test_gp_point_path(torch_dev, orc, d, K, family):
    import torch
    from paper_2210_14313_amd import native, workloads as W
    rng = np.random.default_rng(900 + d)
    b = W.single(d, d + K, "gp", family, W.draw_params(rng, family, d))
    say("case gp points", d, K, family)
    r = orc.smolyak_points(d, d + K, "gp", family, b.param_slice(0))
    prm = torch.as_tensor(b.param_slice(0), dtype=torch.float64).cuda()
    bound = torch.empty(1, dtype=torch.float64, device="cuda")
    out = native.integrate_points(b.problems[0], prm, bound=bound)
    torch.cuda.synchronize()
    err = abs(out.item() - r["q"])
    assert err <= bound.item() + 8 * 2.0 ** -64 * (r["A"] + abs(r["fc"])), (out.item(), r["q"], bound.item())


def test_gp_block_variant(torch_dev, orc):
    import torch
    from oracle import blocked as OB
    from paper_2210_14313_amd import api, native, workloads as W
    b = W.random_small(88, 16, d_range=(5, 40), k_range=(1, 6), rules=("gp",))
    say("case gp blocked")
    ref = np.array([OB.smolyak_blocked(p.d, p.q, p.rule, p.family, b.param_slice(i), 5)
                    for i, p in enumerate(b.problems)])
    params = api.params_tensor(b)
    plan = native.Plan(b.problems, "fp64", block_dims=5)
    try:
        out = torch.empty(len(b), dtype=torch.float64, device="cuda")
        bound = torch.empty_like(out)
        plan.execute(params, out, bound)
        torch.cuda.synchronize()
        got, bnd = out.cpu().numpy(), bound.cpu().numpy()
    finally:
        plan.close()
    assert np.max(np.abs(got - ref) / _scale(b, ref)) <= 1e-12
    assert np.all(np.abs(got - ref) <= bnd)
