"""GPU parity of the gaussian family exp(sum c_i (x_i - u_i)^2) on the
forward sweep ((4.1)-(4.3)): batched plans in the three precision modes,
large and negative c (the growing exp(5 x^2) of (4.1) is c = 20 on the unit
cube), K up to 8, mixed batches, the block variant, and the reverse sweep;
against the oracle's factorised and point-by-point sums and its binary128
factorised gradient.

Tolerances: FP64 within 1e-12 relative and within the stated bound; FP32
modes within the stated bound (their node values are FP64 values rounded
once, like product-peak's).  Gradients: per problem, relative to its
largest entry, 1e-11 in FP64 and 1e-6 with FP32 forward surpluses, the
reverse sweep's bars for the other families.
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


def _run(batch, precision, block_dims=0):
    from paper_2210_14313_amd import api
    vals, bnd = api.integrate(batch, precision, with_bound=True, block_dims=block_dims)
    return vals.cpu().numpy(), bnd.cpu().numpy()


def _check(got, bnd, ref, precision):
    assert np.all(np.abs(got - ref) <= bnd), (precision, np.max(np.abs(got - ref) / np.maximum(bnd, 1e-300)))
    if precision == "fp64":
        assert np.max(np.abs(got - ref) / np.abs(ref)) <= 1e-12


@pytest.mark.parametrize("seed", [1, 2])
def test_gaussian_small_random(torch_dev, orc, seed):
    from paper_2210_14313_amd import workloads as W
    b = W.random_small(600 + seed, 48, d_range=(1, 12), k_range=(0, 6), families=("gaussian",),
                       rules=W.ALL_RULES)
    say("case gaussian small", seed)
    ref = np.array([orc.smolyak_points(p.d, p.q, p.rule, p.family, b.param_slice(i))["q"]
                    for i, p in enumerate(b.problems)])
    for prec in ("fp64", "fp32c", "fp32e"):
        got, bnd = _run(b, prec)
        _check(got, bnd, ref, prec)


@pytest.mark.parametrize("d,K,rule,c", [(2, 5, "gp", 20.0), (3, 8, "gp", 20.0), (10, 4, "cc", -2.0),
                                        (100, 3, "gl", -0.3), (257, 2, "cc", 0.05), (40, 8, "gl_paper", -1.0),
                                        (1000, 2, "tr", -0.01)])
def test_gaussian_edges(torch_dev, orc, d, K, rule, c):
    from paper_2210_14313_amd import workloads as W
    rng = np.random.default_rng(d + 10 * K)
    prm = np.concatenate([c * rng.uniform(0.5, 1.0, d), rng.uniform(0.0, 1.0, d)])
    b = W.single(d, d + K, rule, "gaussian", prm)
    say("case gaussian edge", d, K, rule, c)
    ref = orc.batch_factorised(b)
    for prec in ("fp64", "fp32c", "fp32e"):
        got, bnd = _run(b, prec)
        _check(got, bnd, ref, prec)


def test_gaussian_in_mixed_batch(torch_dev, orc):
    from paper_2210_14313_amd import workloads as W
    b = W.concat([W.random_small(700, 40, d_range=(1, 60), k_range=(0, 6), families=("gaussian",)),
                  W.random_small(701, 40, d_range=(1, 60), k_range=(0, 6))])
    say("case gaussian mixed")
    ref = orc.batch_factorised(b)
    for prec in ("fp64", "fp32c"):
        got, bnd = _run(b, prec)
        assert np.all(np.abs(got - ref) <= bnd), prec


def test_gaussian_block_variant(torch_dev, orc):
    from oracle import blocked as OB
    from paper_2210_14313_amd import workloads as W
    rng = np.random.default_rng(77)
    d = 100
    prm = np.concatenate([rng.uniform(-2.0, 1.0, d) * 0.2, rng.uniform(0.0, 1.0, d)])
    b = W.single(d, d + 4, "gp", "gaussian", prm)
    say("case gaussian blocked")
    ref = np.array([OB.smolyak_blocked(d, d + 4, "gp", "gaussian", prm, 10)])
    got, bnd = _run(b, "fp64", block_dims=10)
    _check(got, bnd, ref, "fp64")


def _grad(batch, precision):
    import torch
    from paper_2210_14313_amd import api, native
    params = api.params_tensor(batch)
    plan = native.Plan(batch.problems, precision)
    try:
        g = plan.execute_grad(params, torch.ones(len(batch), dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        return g.cpu().numpy()
    finally:
        plan.close()


@pytest.mark.parametrize("seed", [1, 2])
def test_gaussian_gradient(torch_dev, orc, seed):
    # gaussian problems of every rule with K up to 8 (compiled and
    # table-driven levels) in one batch with the other sweep families, so
    # the gaussian instantiation of the reverse sweep runs all of them;
    # per problem, error relative to its largest gradient entry
    from paper_2210_14313_amd import workloads as W
    b = W.concat([W.random_small(800 + seed, 24, d_range=(1, 80), k_range=(0, 8), families=("gaussian",),
                                 rules=W.ALL_RULES),
                  W.random_small(810 + seed, 16, d_range=(1, 80), k_range=(0, 6))])
    say("case gaussian gradient", seed)
    ref = np.zeros_like(b.params)
    for i, p in enumerate(b.problems):
        ref[p.param_offset:p.param_offset + W.n_params(p.family, p.d)] = \
            orc.smolyak_factorised_grad(p.d, p.q, p.rule, p.family, b.param_slice(i))
    for prec, tol in (("fp64", 1e-11), ("fp32c", 1e-6)):
        got = _grad(b, prec)
        errs = []
        for i, p in enumerate(b.problems):
            sl = slice(p.param_offset, p.param_offset + W.n_params(p.family, p.d))
            errs.append(np.max(np.abs(got[sl] - ref[sl])) / max(np.max(np.abs(ref[sl])), 1e-300))
        say(prec, "max per-problem relative gradient error", max(errs))
        assert max(errs) <= tol, (prec, int(np.argmax(errs)), max(errs))
