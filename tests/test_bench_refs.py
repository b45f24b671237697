"""The benchmark's stored accuracy references (tests/golden/bench_refs.npz,
written by tests/golden/make_bench_refs.py) agree with the oracle on a
sample of every array, so that a stale file fails here, not in a GPU run."""
import os

import numpy as np
import pytest

from oracle import blocked as OB
from oracle import reference as R
from paper_2210_14313_amd import workloads as W

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "bench_refs.npz")


@pytest.fixture(scope="module")
def refs():
    with np.load(PATH) as z:
        return {k: z[k] for k in z.files}


def test_uneven_batch_values(orc, refs):
    b = W.batched_uneven(4096)
    assert refs["uneven_4096"].shape == (4096,)
    idx = list(range(0, 4096, 97))
    sub = b.subset(idx)
    np.testing.assert_array_equal(orc.batch_factorised(sub), refs["uneven_4096"][idx])


def test_blocked_values(orc, refs):
    b = W.batched_uneven(4096)
    ref = refs["blocked_m10_first256"]
    assert ref.shape == (256,)
    for i in (0, 1, 77, 255):
        p = b.problems[i]
        assert OB.smolyak_blocked(p.d, p.q, p.rule, p.family, b.param_slice(i), 10) == ref[i]


def test_table_4_9_values(refs):
    names = [str(x) for x in refs["table_4_9_names"]]
    assert names == ["exp_alt_d1000", "peak_06_d300"]
    d = 300
    prm = np.concatenate([np.full(d, 1 / 0.45), np.full(d, 0.8)])
    assert float(R.exact("product_peak", d, prm)) == refs["table_4_9_exact"][1]
    assert OB.smolyak_blocked(d, d + 8, "gl_paper", "product_peak", prm, 10) == refs["table_4_9_blocked"][1]


def test_gradient_rows(orc, refs):
    gb = W.gradient_osc_d200()
    g = refs["gradient_osc_d200_first64"]
    assert g.shape == (64, 201)
    for i in (0, 31, 63):
        p = gb.problems[i]
        np.testing.assert_array_equal(orc.smolyak_factorised_grad(p.d, p.q, p.rule, p.family, gb.param_slice(i)),
                                      g[i])


def test_oscillatory_quadratic_value(orc, refs):
    np.testing.assert_array_equal(orc.batch_factorised(W.oscillatory_quadratic_d1000()), refs["oscq_d1000"])


def test_accuracy_scales(orc, refs):
    b = W.batched_uneven(4096)
    idx = list(range(3, 4096, 89))
    sub = b.subset(idx)
    np.testing.assert_allclose(orc.accuracy_scale(sub, refs["uneven_4096"][idx]), refs["uneven_4096_scale"][idx],
                               rtol=1e-15)
    osc = np.array([p.family == "oscillatory" for p in b.problems])
    # the modulus is at least |Q|, with equality for the other family
    s, r = refs["uneven_4096_scale"], refs["uneven_4096"]
    assert np.all(s[osc] >= np.abs(r[osc])) and np.array_equal(s[~osc], np.abs(r[~osc]))
    ob = W.oscillatory_quadratic_d1000()
    np.testing.assert_allclose(orc.accuracy_scale(ob, refs["oscq_d1000"]), refs["oscq_d1000_scale"], rtol=1e-15)
    pd = W.precision_d100()
    np.testing.assert_allclose(orc.accuracy_scale(pd, orc.batch_factorised(pd)), refs["precision_d100_scale"],
                               rtol=1e-15)
    bs = refs["blocked_m10_first256_scale"]
    for i in (0, 1, 77, 255):
        p = b.problems[i]
        if p.family == "oscillatory":
            prm = np.array(b.param_slice(i), copy=True)
            prm[0] -= 0.25
            exp = np.hypot(refs["blocked_m10_first256"][i], OB.smolyak_blocked(p.d, p.q, p.rule, p.family, prm, 10))
        else:
            exp = abs(refs["blocked_m10_first256"][i])
        assert abs(bs[i] - exp) <= 1e-15 * exp
