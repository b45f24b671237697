"""Write the benchmark's accuracy references to tests/golden/bench_refs.npz.

Calls only the CPU oracle, on the seeded workloads the benchmark times, so
that bench.py states its accuracy without running the oracle itself:

* uneven_4096: binary128 factorised values of the 4096-integrand uneven
  batch (d ~ U{8..256}, q - d ~ U{2..6}, Clenshaw-Curtis / Gauss-Legendre,
  oscillatory / exp-sum);
* blocked_m10_first256: the block variant's value (Algorithm 3.3 with step
  m = 10, read as a tensor product of 10-dimensional sparse grids) of the
  first 256 integrands of that batch;
* table_4_9_exact, table_4_9_blocked: exact integrals and block-variant
  values of the m = 10 setting of Table 4.9 (Gauss-Legendre with n_l = l,
  excess K = 8): exp(sum (-1)^(i+1) x_i) on [-1,1]^1000 and
  prod 1/(0.9^2 + (x_i - 0.6)^2) on [-1,1]^300, mapped to the unit cube;
* gradient_osc_d200_first64: binary128 factorised gradients of the first
  64 integrands of the 256-integrand oscillatory d = 200, q = 205
  Clenshaw-Curtis batch (row i: dQ_i/dw, dQ_i/da_1..a_200);
* oscq_d1000: binary128 factorised value of the oscillatory quadratic
  cos(2 pi w + sum a_i (x_i - u_i)^2), d = 1000, q = 1004, Gauss-Patterson
  (workloads.oscillatory_quadratic_d1000);
* *_scale: the oracle's accuracy scale of each value above (|Q|; for the
  oscillatory families the modulus sqrt(Q(w)^2 + Q(w - 1/4)^2) of the
  complex rule, from oracle.accuracy_scale or, for the block rule, the block
  rule at w - 1/4), and precision_d100_scale for the d = 100, q = 105
  Clenshaw-Curtis workload of oracle_full_size.json.

Run from the repository root:  python tests/golden/make_bench_refs.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import blocked as OB  # noqa: E402
from oracle import reference as R  # noqa: E402
from paper_2210_14313_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bench_refs.npz")

#: the Table 4.9 integrands on the unit cube: name, family, d, parameters
TABLE_4_9 = (
    ("exp_alt_d1000", "exp_sum", 1000, lambda d: np.array([2.0 * (-1) ** i for i in range(d)])),
    ("peak_06_d300", "product_peak", 300, lambda d: np.concatenate([np.full(d, 1 / 0.45), np.full(d, 0.8)])),
)
TABLE_4_9_K = 8
BLOCK_M = 10
BLOCKED_CHECK = 256
GRAD_CHECK = 64


def main():
    nthreads = int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))
    batch = W.batched_uneven(4096)
    uneven = oracle.batch_factorised(batch, nthreads=nthreads)
    print("uneven_4096 done", flush=True)
    blocked = np.array([OB.smolyak_blocked(batch.problems[i].d, batch.problems[i].q, batch.problems[i].rule,
                                           batch.problems[i].family, batch.param_slice(i), BLOCK_M)
                        for i in range(BLOCKED_CHECK)])
    print("blocked_m10_first256 done", flush=True)
    t_exact, t_blk = [], []
    for name, fam, d, mk in TABLE_4_9:
        prm = mk(d)
        t_exact.append(float(R.exact(fam, d, prm)))
        t_blk.append(OB.smolyak_blocked(d, d + TABLE_4_9_K, "gl_paper", fam, prm, BLOCK_M))
    print("table_4_9 done", flush=True)
    gb = W.gradient_osc_d200()
    grads = np.stack([oracle.smolyak_factorised_grad(p.d, p.q, p.rule, p.family, gb.param_slice(i))
                      for i, p in enumerate(gb.problems[:GRAD_CHECK])])
    print("gradient_osc_d200_first64 done", flush=True)
    ob = W.oscillatory_quadratic_d1000()
    oscq = oracle.batch_factorised(ob)
    print("oscq_d1000 done", flush=True)
    uneven_scale = oracle.accuracy_scale(batch, uneven, nthreads)
    blocked_scale = np.abs(blocked)
    for i in range(BLOCKED_CHECK):
        p = batch.problems[i]
        if p.family in oracle.OSCILLATORY_FAMILIES:
            prm = np.array(batch.param_slice(i), copy=True)
            prm[0] -= 0.25
            blocked_scale[i] = np.hypot(blocked[i], OB.smolyak_blocked(p.d, p.q, p.rule, p.family, prm, BLOCK_M))
    pd = W.precision_d100()
    pref = oracle.batch_factorised(pd)
    print("scales done", flush=True)
    np.savez(OUT, uneven_4096=uneven, blocked_m10_first256=blocked, oscq_d1000=oscq,
             table_4_9_names=np.array([t[0] for t in TABLE_4_9]),
             table_4_9_exact=np.array(t_exact), table_4_9_blocked=np.array(t_blk),
             gradient_osc_d200_first64=grads,
             uneven_4096_scale=uneven_scale, blocked_m10_first256_scale=blocked_scale,
             oscq_d1000_scale=oracle.accuracy_scale(ob, oscq), precision_d100_scale=oracle.accuracy_scale(pd, pref))


if __name__ == "__main__":
    main()
