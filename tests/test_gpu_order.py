"""Queue orders on the GPU: the longest-first order built on the device
(gs_queue_order), its capture in a graph together with the solve, and what
happens when a caller's order is not a permutation."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import to_np  # noqa: E402
from paper_2609_28458_amd import api, inputs  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    api.lib()


def _prob(w):
    return api.make_problem(w["rhs"], w["tableau"], w["y0"], w["theta"], w["t0"], w["t1"],
                            w["rtol"], w["atol"], w.get("t_out"))


def _is_perm(o, n):
    return np.array_equal(np.sort(o), np.arange(n))


@pytest.mark.parametrize("n", [1, 1000, 100_000])
def test_device_order_is_longest_first_by_the_cost_model(n):
    """The built-in model of the log halo is the host model of
    inputs.predicted_cost (dynamical times in the span, rtol^(-1/5)); the
    device order must be a permutation whose host-model keys never rise by
    more than the bucket width (1/65,534 of the key range)."""
    w = inputs.orbits_uneven(n=n, seed=81)
    sol = api.Solution(_prob(w), api.Launch())
    order = sol.queue_order().cpu().numpy()
    torch.cuda.synchronize()
    assert _is_perm(order, n)
    key = np.log(inputs.predicted_cost(w))[order]
    width = (key.max() - key.min()) / 65534 if n > 1 else 0.0
    assert np.all(np.diff(key) <= width * (1 + 1e-9) + 1e-12)


def test_device_order_of_caller_costs_and_nonfinite_keys():
    n = 5000
    rng = np.random.default_rng(3)
    cost = rng.normal(size=n)
    cost[[7, 11]] = np.nan
    cost[13] = np.inf
    w = inputs.orbits_uneven(n=n, seed=82)
    sol = api.Solution(_prob(w), api.Launch())
    order = sol.queue_order(cost=torch.as_tensor(cost, device="cuda")).cpu().numpy()
    assert _is_perm(order, n)
    assert set(order[-3:]) == {7, 11, 13}       # non-finite keys last
    k = cost[order[:-3]]
    width = (k.max() - k.min()) / 65534
    assert np.all(np.diff(k) <= width * (1 + 1e-9))


def test_solution_does_not_depend_on_the_order():
    """The device order (whose within-bucket order is not fixed) gives the
    same results, bit for bit, as index order."""
    w = inputs.orbits_uneven(n=20_000, seed=83)
    prob = _prob(w)
    ref = to_np(api.solve(prob))
    sol = api.Solution(prob, api.Launch(block=128, wide=256))
    sol.queue_order()
    sol.run()
    torch.cuda.synchronize()
    got = to_np(sol)
    for k in ref:
        np.testing.assert_array_equal(got[k], ref[k], err_msg=k)


def test_order_and_solve_captured_in_one_graph():
    """Order build and solve captured together; every replay (with eager
    work and synchronisations between them) equals the eager result."""
    w = inputs.orbits_uneven(n=30_000, seed=84)
    prob = _prob(w)
    ref = to_np(api.solve(prob))
    sol = api.Solution(prob, api.Launch(block=128, wide=256))
    sol.queue_order()  # allocates the order and its workspace outside the capture

    def body(stream):
        sol.queue_order(stream=stream)
        sol.run(stream=stream)

    g = api.Captured(body)
    for rep in range(4):
        sol.y_final.fill_(-1.0)
        sol.status.fill_(-1)
        x = torch.randn(1000, 1000, device="cuda", dtype=torch.float64)
        _ = (x @ x).sum().item()          # eager work between replays
        g.launch()
        torch.cuda.synchronize()
        got = to_np(sol)
        for k in ref:
            np.testing.assert_array_equal(got[k], ref[k], err_msg=f"replay {rep}: {k}")
        assert _is_perm(sol.order.cpu().numpy(), prob.n)


def test_non_permutation_orders():
    """The binding refuses an order that is not a permutation; passed
    unchecked, the index it misses is reported as NOT_RUN by the solve and
    gets NaN cotangents from the adjoint, and every other trajectory is
    solved exactly as in index order."""
    w = inputs.orbits_forward(n=300, seed=85)
    prob = _prob(w)
    bad = np.arange(300)
    bad[17] = 18                                    # 18 twice, 17 missing
    sol = api.Solution(prob, api.Launch(ckpt_every=1, ckpt_capacity=4000))
    with pytest.raises(ValueError):
        sol.set_order(bad)
    with pytest.raises(ValueError):
        sol.set_order(np.arange(299))
    sol.set_order(bad, check=False)
    sol.run()
    ref = to_np(api.solve(prob))
    got = to_np(sol)
    assert got["status"][17] == 6                   # GS_TRAJ_NOT_RUN
    keep = np.arange(300) != 17
    assert np.all(got["status"][keep] == 0)
    np.testing.assert_array_equal(got["y_final"][:, keep], ref["y_final"][:, keep])
    yb = torch.ones((1, 6, 300), dtype=torch.float64, device="cuda")
    y0b, thb = api.solve_vjp(sol, ybar_final=yb)
    torch.cuda.synchronize()
    y0b, thb = y0b.cpu().numpy(), thb.cpu().numpy()
    assert np.all(np.isnan(y0b[0, :, 17])) and np.all(np.isnan(thb[0, :, 17]))
    assert np.all(np.isfinite(y0b[0][:, keep])) and np.all(np.isfinite(thb[0][:, keep]))
    # out-of-range entries are skipped the same way
    oob = np.arange(300)
    oob[5] = 10_000
    s2 = api.Solution(prob, api.Launch())
    s2.set_order(oob, check=False)
    s2.run()
    st = s2.status.cpu().numpy()
    assert st[5] == 6 and np.all(st[np.arange(300) != 5] == 0)


def test_forward_sensitivities_take_a_device_order():
    w = inputs.orbits_uneven(n=4000, seed=86)
    prob = _prob(w)
    ref_sol, ref_S, _ = api.solve_sens(prob, [6, 7])
    sol = api.Solution(prob, api.Launch())
    order = sol.queue_order()
    got_sol, got_S, _ = api.solve_sens(prob, [6, 7], order=order)
    torch.cuda.synchronize()
    assert torch.equal(got_S, ref_S)
    assert torch.equal(got_sol.y_final, ref_sol.y_final)


def test_pilot_fitted_cost_ranks_the_precession_binaries():
    """autotune.pilot_cost on 20,000 binaries: a pilot solve of a sample over
    the last decade of separation and a least-squares fit on log q, the spin
    magnitudes and the three cosines; the fitted cost ranks the full solve's
    attempts with a rank correlation above 0.9, and the device order built
    from it is a permutation."""
    from scipy.stats import spearmanr

    from paper_2609_28458_amd import autotune

    w = inputs.spin_precession(n=20_000, seed=87)
    w.update(t_out=None)
    prob = _prob(w)
    pilot = _prob({**w, "t0": 100.0 ** -0.5})
    y, th = pilot.y0, pilot.theta
    feats = torch.stack([torch.log(th[0]), th[1], th[2], (y[0:3] * y[3:6]).sum(0),
                         (y[0:3] * y[6:9]).sum(0), (y[3:6] * y[6:9]).sum(0)])
    cost = autotune.pilot_cost(pilot, feats, sample=2048).contiguous()
    sol = api.Solution(prob, api.Launch())
    order = sol.queue_order(cost).cpu().numpy()
    sol.run()
    torch.cuda.synchronize()
    assert _is_perm(order, prob.n)
    att = (sol.n_accepted + sol.n_rejected).cpu().numpy()
    rho = spearmanr(cost.cpu().numpy(), att).correlation
    assert rho > 0.9, rho
