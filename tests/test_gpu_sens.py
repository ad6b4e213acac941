"""Forward sensitivities on the GPU (gs_solve_sens): eq:sens carried through
the stages (eq:stage-sens) in the same launch as the solution.

The solution is the plain solve's, bit for bit (step control reads values
only); the tangents are the oracle's forward sensitivities of the same
discrete solution, at the output nodes and at t1, up to rounding.
"""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import gpu_solve, oracle_solve, to_np  # noqa: E402
from parity_log import record  # noqa: E402
from paper_2609_28458_amd import api, inputs  # noqa: E402
from test_gpu_forward import CASES  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    api.lib()


def _prob(w):
    return api.make_problem(w["rhs"], w["tableau"], w["y0"], w["theta"], w["t0"], w["t1"],
                            w["rtol"], w["atol"], w.get("t_out"))


def _close(got, ref, tol=1e-9, name="sensitivities vs oracle"):
    # relative to the largest sensitivity of the trajectory (floor 1)
    scale = np.maximum(np.abs(ref).reshape(-1, ref.shape[-1]).max(axis=0), 1.0)
    err = np.abs(got - ref) / scale
    record(name, err.max(), tol)
    assert err.max() < tol, err.max()


@pytest.mark.parametrize("tab", ["dopri5", "tsit5", "verner7"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_sensitivities_match_oracle(orc, name, make, tab):
    w = {**make(150), "tableau": tab}
    prob = _prob(w)
    d, p = prob.d, api.NPARAM[prob.rhs]
    cols = [0, d + p - 1, d - 1]  # an initial condition, a parameter, another state; 2 launches
    sol, S_final, S_out = api.solve_sens(prob, cols)
    torch.cuda.synchronize()
    g = to_np(sol)
    ref = to_np(gpu_solve(w))
    for k in ref:
        np.testing.assert_array_equal(g[k], ref[k], err_msg=k)
    assert np.all(g["status"] == 0)
    o = oracle_solve(orc, w, sens_cols=cols)
    np.testing.assert_array_equal(g["n_accepted"], o["n_accepted"])
    _close(S_final.cpu().numpy(), o["S_final"], name=f"sens vs oracle {name} {tab} final")
    if S_out is not None:
        _close(S_out.cpu().numpy(), o["S_out"], name=f"sens vs oracle {name} {tab} outputs")



def _same_sens(prob, cols, launch, order=None):
    """Solution, outputs and tangents of `launch` against the same launch
    with one lane per trajectory."""
    ref, Sf, So = api.solve_sens(prob, cols, dataclasses.replace(launch, wide=0), order=order)
    got, Gf, Go = api.solve_sens(prob, cols, launch, order=order)
    torch.cuda.synchronize()
    r, g = to_np(ref), to_np(got)
    for k in r:
        np.testing.assert_array_equal(g[k], r[k], err_msg=k)
    np.testing.assert_array_equal(Gf.cpu().numpy(), Sf.cpu().numpy(), err_msg="S_final")
    if So is not None:
        np.testing.assert_array_equal(Go.cpu().numpy(), So.cpu().numpy(), err_msg="S_out")
    return r


@pytest.mark.parametrize("tab", ["dopri5", "tsit5", "verner7"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_wide_group_sensitivities_equal_single_lanes(name, make, tab):
    """Sensitivities on 16-lane groups (the head of the queue, then every
    trajectory), with output nodes and with the final state only: the
    solution, the outputs and every tangent bitwise those of one lane per
    trajectory (a group gathers its dual stage point and evaluates the
    ordinary right-hand side; Verner 7 takes its shortened-step outputs on
    the group)."""
    w = {**make(150), "tableau": tab}
    for ww in (w, {**w, "t_out": None}):
        prob = _prob(ww)
        d, p = prob.d, api.NPARAM[prob.rhs]
        cols = [0, d + p - 1, d - 1]  # two launches, two columns then one
        for wide in (37, prob.n):
            r = _same_sens(prob, cols, api.Launch(wide=wide))
        assert np.all(r["status"] == 0)


@pytest.mark.parametrize("tab", ["dopri5", "verner7"])
def test_wide_group_sensitivities_of_stopped_trajectories(tab):
    """A step limit stops most trajectories: NaN outputs and tangents past
    the stop, statuses and counts, bitwise those of one lane each; a
    longest-first order puts the longest on the groups; outputs also in the
    [K][n][d] layout."""
    w = {**inputs.orbits_forward(200, seed=55), "tableau": tab}
    prob = _prob(w)
    order = np.argsort(-inputs.predicted_cost(w), kind="stable")
    for L in (dict(), dict(max_steps=120), dict(out_layout="knd")):
        r = _same_sens(prob, [6, 7], api.Launch(wide=64, **L), order=order)
        if "max_steps" in L:
            assert np.any(r["status"] != 0)

def test_sensitivities_of_the_gradient_workload(orc):
    """100,000 orbits to t = 100 with the two halo parameters (v0, q) as
    columns, the paper's stream-gradient setting: sampled against the
    oracle."""
    w = inputs.orbits_gradient()
    prob = _prob(w)
    sol, S_final, _ = api.solve_sens(prob, [6, 7])
    torch.cuda.synchronize()
    assert bool((sol.status == 0).all())
    idx = np.sort(np.random.default_rng(21).choice(prob.n, 200, replace=False))
    o = oracle_solve(orc, w, idx, sens_cols=[6, 7])
    np.testing.assert_array_equal(sol.n_accepted.cpu().numpy()[idx], o["n_accepted"])
    _close(S_final.cpu().numpy()[:, :, idx], o["S_final"], name="sens vs oracle, gradient workload sample")
    # the launch the benchmark times: longest first, the longest 256 on
    # 16-lane groups; bitwise the single-lane result, the 50 longest checked
    # against the oracle as well
    order = api.Solution(prob, api.Launch()).queue_order().clone()
    g, G_final, _ = api.solve_sens(prob, [6, 7], api.Launch(wide=256), order=order)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(G_final.cpu().numpy(), S_final.cpu().numpy())
    np.testing.assert_array_equal(g.y_final.cpu().numpy(), sol.y_final.cpu().numpy())
    top = np.sort(np.argsort(-sol.n_accepted.cpu().numpy(), kind="stable")[:50])
    o = oracle_solve(orc, w, top, sens_cols=[6, 7])
    _close(G_final.cpu().numpy()[:, :, top], o["S_final"],
           name="sens vs oracle, gradient workload, 50 longest on groups")
