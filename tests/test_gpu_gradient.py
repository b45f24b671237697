"""GPU parity of the reverse sweep (gradient of every result with respect to
every parameter) against the oracle's binary128 factorised gradient, central
finite differences of the FP64 forward pass, and closed-form gradients."""
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
    return torch


def _grad(batch, precision, gout=None):
    import torch
    from paper_2210_14313_amd import api, native
    params = api.params_tensor(batch)
    plan = native.Plan(batch.problems, precision)
    if gout is None:
        gout = torch.ones(len(batch), dtype=torch.float64, device="cuda")
    g = plan.execute_grad(params, gout)
    torch.cuda.synchronize()
    plan.close()
    return g.cpu().numpy()


def _oracle_grad(orc, batch, weights=None):
    g = np.zeros_like(batch.params)
    for i, p in enumerate(batch.problems):
        gi = orc.smolyak_factorised_grad(p.d, p.q, p.rule, p.family, batch.param_slice(i))
        w = 1.0 if weights is None else weights[i]
        g[p.param_offset:p.param_offset + len(gi)] = w * gi
    return g


def _per_problem_err(batch, got, ref):
    from paper_2210_14313_amd import workloads as W
    errs = []
    for i, p in enumerate(batch.problems):
        sl = slice(p.param_offset, p.param_offset + W.n_params(p.family, p.d))
        scale = max(np.max(np.abs(ref[sl])), 1e-300)
        errs.append(np.max(np.abs(got[sl] - ref[sl])) / scale)
    return np.array(errs)


def test_gradient_workload_vs_oracle(torch_dev, orc):
    from paper_2210_14313_amd import workloads as W
    b = W.gradient_osc_d200()
    say("case gradient_osc_d200 adjoint")
    ref = _oracle_grad(orc, b)
    got = _grad(b, "fp64")
    err = _per_problem_err(b, got, ref)
    assert np.max(err) <= 1e-12, (int(np.argmax(err)), float(np.max(err)))
    got32 = _grad(b, "fp32c")
    err32 = _per_problem_err(b, got32, ref)
    assert np.max(err32) <= 1e-6, float(np.max(err32))


def test_gradient_matches_closed_form(torch_dev):
    from oracle import reference as R
    from paper_2210_14313_amd import workloads as W
    b = W.gradient_osc_d200(n=4)
    say("case closed-form gradient")
    got = _grad(b, "fp64")
    for i, p in enumerate(b.problems):
        ge = R.exact_grad_oscillatory(b.param_slice(i)[0], b.param_slice(i)[1:])
        gi = got[p.param_offset:p.param_offset + p.d + 1]
        assert np.max(np.abs(gi - ge)) <= 1e-11 * np.max(np.abs(ge))


def test_gradient_matches_central_differences(torch_dev):
    import torch
    from paper_2210_14313_amd import api, native, workloads as W
    b = W.random_small(31, 12, d_range=(2, 70), k_range=(1, 5), families=("exp_sum", "oscillatory", "product_peak"))
    params = api.params_tensor(b)
    plan = native.Plan(b.problems, "fp64")
    g = plan.execute_grad(params, torch.ones(len(b), dtype=torch.float64, device="cuda")).cpu().numpy()
    say("case central differences")
    owner = np.zeros(len(b.params), dtype=int)
    for i, p in enumerate(b.problems):
        owner[p.param_offset:p.param_offset + W.n_params(p.family, p.d)] = i
    rng = np.random.default_rng(0)
    for k in sorted(rng.choice(len(b.params), 40, replace=False)):
        i = owner[k]
        h = 1e-4 * max(1.0, abs(float(b.params[k])))
        vals = []
        for step in (2, 1, -1, -2):
            pk = params.clone()
            pk[k] += step * h
            vals.append(plan.execute(pk)[i].item())
        # fourth-order central difference
        fd = (-vals[0] + 8 * vals[1] - 8 * vals[2] + vals[3]) / (12 * h)
        scale = max(abs(g[k]), 1e-3 * abs(plan.execute(params)[i].item()), 1e-12)
        assert abs(fd - g[k]) <= 1e-7 * scale + 1e-9, (k, fd, g[k])
    plan.close()


@pytest.mark.parametrize("seed", [41, 42])
def test_gradient_small_random_all_families(torch_dev, orc, seed):
    from paper_2210_14313_amd import workloads as W
    # d up to 600: several waves per integrand and several coordinates per lane
    b = W.random_small(seed, 40, d_range=(1, 600), k_range=(0, 5))
    say("case gradient random", seed)
    ref = _oracle_grad(orc, b)
    w = np.random.default_rng(seed).normal(size=len(b))
    import torch
    got = _grad(b, "fp64", torch.as_tensor(w, dtype=torch.float64).cuda())
    ref = _oracle_grad(orc, b, w)
    err = _per_problem_err(b, got, ref)
    assert np.max(err) <= 1e-11, (int(np.argmax(err)), float(np.max(err)))


def test_autograd_function(torch_dev):
    import torch
    from paper_2210_14313_amd import api, native, workloads as W
    b = W.random_small(7, 10, d_range=(3, 90), k_range=(1, 4), families=("exp_sum", "oscillatory"))
    params = api.params_tensor(b).requires_grad_(True)
    plan = native.Plan(b.problems, "fp64")
    say("case autograd")
    q = api.SGIntegral.apply(params, plan)
    w = torch.linspace(0.5, 1.5, len(b), dtype=torch.float64, device="cuda")
    (q * w).sum().backward()
    ref = plan.execute_grad(params.detach(), w)
    assert torch.allclose(params.grad, ref, rtol=0, atol=0)
    plan.close()


def test_gradient_rejects_shared_parameters(torch_dev):
    import torch
    from paper_2210_14313_amd import native, workloads as W
    b = W.single(4, 6, "cc", "exp_sum", np.ones(4))
    probs = [b.problems[0], W.Problem(4, 6, "cc", "exp_sum", 0)]
    plan = native.Plan(probs, "fp64")
    params = torch.ones(4, dtype=torch.float64, device="cuda")
    with pytest.raises(native.SgError) as e:
        plan.execute_grad(params, torch.ones(2, dtype=torch.float64, device="cuda"))
    assert e.value.status == 1
    plan.close()
