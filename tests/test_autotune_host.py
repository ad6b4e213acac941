"""Host logic of the autotuner that needs no GPU: the subset of a problem a
pilot solve runs on."""
import numpy as np
import pytest
import torch

from paper_2609_28458_amd import api, autotune


def _prob(n, theta_shared, t_out):
    f64 = dict(dtype=torch.float64)
    return api.Problem(
        2, 1, torch.arange(6 * n, **f64).reshape(6, n),
        torch.arange(3, **f64) if theta_shared else torch.arange(3 * n, **f64).reshape(3, n),
        torch.zeros(1, **f64), torch.arange(n, **f64) + 1.0, torch.full((n,), 1e-6, **f64),
        torch.full((1,), 1e-8, **f64), t_out)


@pytest.mark.parametrize("shared", [True, False])
def test_subset_slices_by_role(shared):
    # n = 3 equals p = 3 and K = 3: lengths alone could not tell shared from per-trajectory
    t_out = torch.tensor([0.5, 1.0, 1.5], dtype=torch.float64)
    p = _prob(3, shared, t_out)
    idx = torch.tensor([2, 0])
    q = autotune._subset(p, idx)
    assert torch.equal(q.y0, p.y0[:, [2, 0]])
    assert torch.equal(q.theta, p.theta if shared else p.theta[:, [2, 0]])
    assert torch.equal(q.t1, p.t1[[2, 0]]) and torch.equal(q.rtol, p.rtol[[2, 0]])
    assert torch.equal(q.t0, p.t0) and torch.equal(q.atol, p.atol)
    assert torch.equal(q.t_out, t_out)
    t_out2 = torch.arange(6, dtype=torch.float64).reshape(2, 3)
    q2 = autotune._subset(_prob(3, shared, t_out2), idx)
    assert torch.equal(q2.t_out, t_out2[:, [2, 0]])


def test_pilot_order_rejects_bad_features():
    p = _prob(4, True, None)
    with pytest.raises(ValueError):
        autotune.pilot_order(p, [np.array([1.0, np.inf, 0.0, 2.0])])
    with pytest.raises(ValueError):
        autotune.pilot_order(p, [np.ones(3)])
