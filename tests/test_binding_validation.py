"""The Python binding checks every tensor before the C ABI sees its raw
pointer (CPU only: the checks run before any context or launch)."""
import numpy as np
import pytest
import torch

from paper_2210_14313_amd import native, workloads as W


def test_n_params_matches_the_workload_layout():
    for fam in list(W.FAMILIES) + list(W.POINT_ONLY_FAMILIES) + list(W.EXTRA_SWEEP_FAMILIES):
        for d in (1, 7, 300):
            assert native.n_params(fam, d) == W.n_params(fam, d), (fam, d)


def test_param_extent_is_the_batch_extent():
    b = W.random_small(3, 40, d_range=(1, 30), k_range=(0, 4))
    assert native.param_extent(b.problems) == len(b.params)
    sub = b.subset([5, 2, 9])
    assert native.param_extent(sub.problems) == len(sub.params)


def test_check_tensor_rejects_what_the_abi_cannot_bound():
    ok_cpu = torch.zeros(8, dtype=torch.float64)
    with pytest.raises(ValueError, match="device"):
        native.check_tensor("params", ok_cpu, 8)              # host memory
    with pytest.raises(ValueError, match="tensor"):
        native.check_tensor("params", np.zeros(8), 8)        # not a tensor
    with pytest.raises(ValueError):
        native.check_tensor("params", torch.zeros(8, dtype=torch.float32), 8)


def test_one_shot_paths_validate_before_any_context():
    b = W.random_small(4, 1, d_range=(5, 5), k_range=(2, 2), families=("oscillatory",))
    p = b.problems[0]
    host = torch.as_tensor(b.param_slice(0))
    with pytest.raises(ValueError):
        native.integrate_one(p, host, "fp64")
    with pytest.raises(ValueError):
        native.integrate_points(p, host)
