"""sg_integrate_noalloc through the C ABI against sg_integrate (the entry
point it is a variant of): the same kernels and launch shape, so the values
and bounds must agree bit for bit, on two calls in a row, the second with a
smaller input; each also against the oracle (FP64 within 1e-12 of the
oracle's accuracy scale, every result within its stated bound), and no
device memory taken after the first call."""
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


def _free_bytes():
    hip = ctypes.CDLL("libamdhip64.so")
    free, total = ctypes.c_size_t(), ctypes.c_size_t()
    assert hip.hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)) == 0
    return free.value


FAMILIES = ("exp_sum", "oscillatory", "product_peak", "gaussian", "oscillatory_quadratic",
            "oscillatory_quadratic_linear")


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
@pytest.mark.parametrize("family", FAMILIES)
def test_noalloc_matches_integrate_two_calls(torch_dev, orc, family, precision):
    import torch
    from paper_2210_14313_amd import native, workloads as W
    rng = np.random.default_rng(700 + FAMILIES.index(family))
    # the first call splits over 12 workgroups, the second runs on one
    # workgroup (the complex sweep: over 3); product-peak factors near 1 at
    # d = 3000 keep its value in the double range
    cases = [(3000, 3, "cc"), (700, 5, "gl")]
    for call, (d, K, rule) in enumerate(cases):
        prm = W.draw_params(rng, family, d)
        if family == "exp_sum":
            prm = prm / d
        if family == "product_peak" and d > 1000:
            prm = np.concatenate([np.ones(d), rng.uniform(0.4, 0.6, d)])
        b = W.single(d, d + K, rule, family, prm)
        p = b.problems[0]
        pr = torch.as_tensor(prm, dtype=torch.float64).cuda()
        say("case noalloc", family, precision, "call", call, "d", d, "K", K, rule)
        o1 = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        b1 = torch.full_like(o1, float("nan"))
        o2 = torch.full_like(o1, float("nan"))
        b2 = torch.full_like(o1, float("nan"))
        native.integrate_one(p, pr, precision, out=o1, bound=b1)
        native.integrate_noalloc(p, pr, precision, out=o2, bound=b2)
        torch.cuda.synchronize()
        assert o1.item() == o2.item() and b1.item() == b2.item(), (o1.item(), o2.item(), b1.item(), b2.item())
        ref = orc.smolyak_factorised(p.d, p.q, p.rule, p.family, prm)
        scale = orc.accuracy_scale_one(p.d, p.q, p.rule, p.family, prm, ref)
        assert abs(o2.item() - ref) <= b2.item(), (o2.item(), ref, b2.item())
        if precision == "fp64":
            assert abs(o2.item() - ref) <= 1e-12 * scale, (o2.item(), ref)
        elif family in ("exp_sum", "oscillatory"):
            assert abs(o2.item() - ref) <= 1e-7 * scale, (o2.item(), ref)
        elif family.startswith("oscillatory_quadratic"):
            assert abs(o2.item() - ref) <= 1e-6 * scale, (o2.item(), ref)


def test_noalloc_takes_no_device_memory(torch_dev):
    import torch
    from paper_2210_14313_amd import native, workloads as W
    rng = np.random.default_rng(5)
    b = W.single(2000, 2004, "cc", "oscillatory", W.draw_params(rng, "oscillatory", 2000))
    p = b.problems[0]
    pr = torch.as_tensor(b.param_slice(0), dtype=torch.float64).cuda()
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    bound = torch.empty_like(out)
    native.integrate_noalloc(p, pr, "fp64", out=out, bound=bound)   # loads the code object
    torch.cuda.synchronize()
    before = _free_bytes()
    vals = []
    for _ in range(5):
        native.integrate_noalloc(p, pr, "fp64", out=out, bound=bound)
        torch.cuda.synchronize()
        vals.append(out.item())
    assert _free_bytes() == before
    assert len(set(vals)) == 1


def test_noalloc_rejections(torch_dev):
    import torch
    from paper_2210_14313_amd import native, workloads as W
    b = W.single(10, 12, "cc", "exp_sum", np.full(10, 0.1))
    p = b.problems[0]
    pr = torch.as_tensor(b.param_slice(0), dtype=torch.float64).cuda()
    with pytest.raises(ValueError):
        native.integrate_noalloc(p, pr, "fp64")                     # no out given
    bad = W.Problem(10, 9, "cc", "exp_sum", 0)                      # q < d
    with pytest.raises(native.SgError) as e:
        native.integrate_noalloc(bad, pr, "fp64", out=torch.empty(1, dtype=torch.float64, device="cuda"))
    assert e.value.status == 1
