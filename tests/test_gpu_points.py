"""GPU parity of the literal point-by-point path (sg_integrate_points)
against the CPU oracle's point-by-point sum (2.6)-(2.7), against the stored
full-size oracle values, and against the factorised GPU sweep.

Tolerance: both sides evaluate the same sum, the GPU in FP64 with
double-double accumulation, the oracle in x87 extended precision with
Neumaier accumulation.  Each GPU result must lie within the rounding bound
the library states for it plus the oracle's own rounding scale
(8 * 2^-64 * (A + |f(c)|)), and within 1e-12 relative wherever that bound
is below it (relative to the oracle's accuracy scale: |Q|, oscillatory
families the modulus of the complex Smolyak sum); the terms' cancellation puts
the bound far above 1e-12 at d = 100.
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
    from paper_2210_14313_amd import native
    native.lib()
    return torch


def _acc(batch, i, ref):
    import oracle
    p = batch.problems[i]
    return oracle.accuracy_scale_one(p.d, p.q, p.rule, p.family, batch.param_slice(i), ref)


def _points(batch, i, max_points=0, with_bound=False):
    import torch
    from paper_2210_14313_amd import native
    p = batch.problems[i]
    prm = torch.as_tensor(batch.param_slice(i), dtype=torch.float64).cuda()
    bound = torch.empty(1, dtype=torch.float64, device="cuda") if with_bound else None
    out = native.integrate_points(p, prm, bound=bound, max_points=max_points)
    torch.cuda.synchronize()
    return (out.item(), bound.item()) if with_bound else out.item()


def _check(got, bnd, ref, scale, oracle_scale):
    err = abs(got - ref)
    tol_oracle = 8 * 2.0 ** -64 * oracle_scale
    assert err <= bnd + tol_oracle, (got, ref, err, bnd)
    if bnd + tol_oracle <= 1e-12 * scale:
        assert err <= 1e-12 * scale, (got, ref, err)


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_points_small_random_vs_point_oracle(torch_dev, orc, seed):
    from paper_2210_14313_amd import workloads as W
    b = W.random_small(seed, 40, d_range=(1, 12), k_range=(0, 5))
    say("case points small random seed", seed)
    for i, p in enumerate(b.problems):
        r = orc.smolyak_points(p.d, p.q, p.rule, p.family, b.param_slice(i))
        got, bnd = _points(b, i, with_bound=True)
        _check(got, bnd, r["q"], _acc(b, i, r["q"]), r["A"] + abs(r["fc"]))


@pytest.mark.parametrize("d,K,rule,family", [(1, 8, "cc", "exp_sum"), (2, 8, "gl", "oscillatory"),
                                             (7, 0, "tr", "product_peak"), (30, 3, "cc", "product_peak"),
                                             (65, 2, "gl_paper", "oscillatory"), (3, 8, "tr", "product_peak"),
                                             (200, 2, "cc", "exp_sum")])
def test_points_edges_vs_point_oracle(torch_dev, orc, d, K, rule, family):
    from paper_2210_14313_amd import workloads as W
    rng = np.random.default_rng(1000 * d + K)
    b = W.single(d, d + K, rule, family, W.draw_params(rng, family, d))
    say("case points edge", d, K, rule, family)
    r = orc.smolyak_points(d, d + K, rule, family, b.param_slice(0))
    got, bnd = _points(b, 0, with_bound=True)
    _check(got, bnd, r["q"], _acc(b, 0, r["q"]), r["A"] + abs(r["fc"]))


def test_points_plain_exp_d10(torch_dev, orc):
    from paper_2210_14313_amd import workloads as W
    b = W.plain_exp_d10()
    say("case points plain_exp_d10")
    r = orc.smolyak_points(10, 14, "cc", "exp_sum", b.param_slice(0))
    got, bnd = _points(b, 0, with_bound=True)
    _check(got, bnd, r["q"], _acc(b, 0, r["q"]), r["A"] + abs(r["fc"]))
    assert abs(got - r["q"]) <= 1e-12 * abs(r["q"])


def _golden_rows():
    path = os.path.join(GOLDEN, "oracle_full_size.json")
    if not os.path.exists(path):
        return []
    return [r for r in json.load(open(path))["rows"] if r["workload"] == "precision_d100"]


@pytest.mark.parametrize("row", _golden_rows(), ids=lambda r: f"{r['workload']}-{r['index']}")
def test_points_full_size_against_stored_point_oracle(torch_dev, row):
    # d = 100, q = 105, Clenshaw-Curtis: 2.08e10 points
    from paper_2210_14313_amd import workloads as W
    b = W.STANDARD[row["workload"]]().subset([row["index"]])
    p = b.problems[0]
    say("case points full size", row["workload"], row["index"], p.family)
    ref = row["points_hi"] + row["points_lo"]
    got, bnd = _points(b, 0, with_bound=True)
    say("  got", got, "oracle", ref, "bound", bnd)
    _check(got, bnd, ref, _acc(b, 0, ref), row["points_A"] + abs(row["fc"]))


def test_points_agree_with_factorised_sweep(torch_dev):
    import torch
    from paper_2210_14313_amd import api, native, workloads as W
    b = W.random_small(21, 24, d_range=(20, 150), k_range=(1, 4))
    say("case points vs sweep")
    vals, vb = api.integrate(b, "fp64", with_bound=True)
    vals, vb = vals.cpu().numpy(), vb.cpu().numpy()
    for i, p in enumerate(b.problems):
        got, bnd = _points(b, i, with_bound=True)
        assert abs(got - vals[i]) <= bnd + vb[i], (i, p, got, vals[i], bnd, vb[i])


def test_points_deterministic_and_limits(torch_dev):
    import torch
    from paper_2210_14313_amd import native, workloads as W
    b = W.random_small(8, 3, d_range=(40, 60), k_range=(3, 4))
    say("case points determinism")
    for i in range(len(b)):
        assert _points(b, i) == _points(b, i)
    p = b.problems[0]
    npts = native.counts(p.d, p.q, p.rule)[1]
    with pytest.raises(native.SgError) as e:
        _points(b, 0, max_points=npts - 1)
    assert e.value.status == 2
    assert _points(b, 0, max_points=npts) == _points(b, 0)


@pytest.mark.parametrize("d,K,rule", [(1, 8, "gl"), (3, 6, "cc"), (8, 5, "tr"), (12, 4, "gl_paper"), (40, 3, "cc")])
def test_points_corner_peak_vs_point_oracle(torch_dev, orc, d, K, rule):
    # a ridge integrand that does not factor: only the point path handles it
    from paper_2210_14313_amd import workloads as W
    rng = np.random.default_rng(500 + d)
    b = W.single(d, d + K, rule, "corner_peak", W.draw_params(rng, "corner_peak", d))
    say("case points corner peak", d, K, rule)
    r = orc.smolyak_points(d, d + K, rule, "corner_peak", b.param_slice(0))
    got, bnd = _points(b, 0, with_bound=True)
    _check(got, bnd, r["q"], _acc(b, 0, r["q"]), r["A"] + abs(r["fc"]))


def test_points_corner_peak_converges_to_closed_form(torch_dev):
    from oracle import reference as R
    from paper_2210_14313_amd import workloads as W
    rng = np.random.default_rng(9)
    a = W.draw_params(rng, "corner_peak", 3)
    b = W.single(3, 11, "gl", "corner_peak", a)
    say("case points corner peak closed form")
    got = _points(b, 0)
    ex = float(R.exact_corner_peak(a))
    assert abs(got - ex) <= 1e-12 * ex


def test_corner_peak_rejected_by_the_sweep(torch_dev):
    from paper_2210_14313_amd import native, workloads as W
    b = W.single(4, 6, "cc", "corner_peak", np.full(4, 0.25))
    with pytest.raises(native.SgError) as e:
        native.Plan(b.problems, "fp64")
    assert e.value.status == 2


@pytest.mark.parametrize("family", ["gaussian", "oscillatory_quadratic", "oscillatory_quadratic_linear"])
@pytest.mark.parametrize("d,K,rule", [(1, 8, "gp"), (2, 7, "cc"), (5, 5, "gl"), (9, 4, "gp"), (30, 3, "tr"),
                                      (64, 2, "gl_paper")])
def test_points_quadratic_families_vs_point_oracle(torch_dev, orc, family, d, K, rule):
    # the exponentials and sines of quadratics of (4.1)-(4.3)
    from paper_2210_14313_amd import workloads as W
    rng = np.random.default_rng(40 * d + K)
    b = W.single(d, d + K, rule, family, W.draw_params(rng, family, d))
    say("case points quadratic", family, d, K, rule)
    r = orc.smolyak_points(d, d + K, rule, family, b.param_slice(0))
    got, bnd = _points(b, 0, with_bound=True)
    _check(got, bnd, r["q"], _acc(b, 0, r["q"]), r["A"] + abs(r["fc"]))


def test_points_paper_table_4_1_first_row(torch_dev):
    # exp(5 x1^2 + 5 x2^2) on [-1,1]^2 with Gauss-Patterson, accuracy level 6
    # (excess 5): relative error 1.0349e-1
    import mpmath as mp
    from oracle import reference as R
    from paper_2210_14313_amd import workloads as W
    g = json.load(open(os.path.join(GOLDEN, "paper_table_4_1.json")))
    row = g["rows"][0]
    prm = np.array(row["params"], dtype=np.float64)
    b = W.single(row["d"], row["d"] + row["q"] - 1, g["rule"], g["family"], prm)
    say("case points table 4.1")
    got = _points(b, 0)
    ex = R.exact(g["family"], row["d"], prm)
    rel = float(abs((mp.mpf(got) - ex) / ex))
    assert abs(rel - row["rel_err"]) <= 1.01e-5 * 10 ** np.floor(np.log10(row["rel_err"])) * 10, rel


@pytest.mark.parametrize("family", ["corner_peak"])
def test_point_families_rejected_by_plans(torch_dev, family):
    from paper_2210_14313_amd import native, workloads as W
    b = W.single(4, 6, "cc", family, W.draw_params(np.random.default_rng(1), family, 4))
    with pytest.raises(native.SgError) as e:
        native.Plan(b.problems, "fp64")
    assert e.value.status == 2
