"""GPU forward solve vs the oracle on the same seeded inputs.

Parity bar: every output within 1e-9 relative (floor 1) of the oracle at the
same tableau, controller and tolerances, and the same accepted and rejected
step counts (the two take the same steps; only rounding differs).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import gpu_solve, oracle_solve, rel_err, to_np  # noqa: E402
from paper_2609_28458_amd import api, inputs  # noqa: E402

TOL = 1e-9


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    api.lib()


def _check(g, o, idx=None, max_count_mismatch=0):
    sl = slice(None) if idx is None else idx
    bad = np.sum(g["n_accepted"][sl] != o["n_accepted"]) + np.sum(g["n_rejected"][sl] != o["n_rejected"])
    assert bad <= max_count_mismatch, f"{bad} step-count mismatches"
    same = (g["n_accepted"][sl] == o["n_accepted"]) & (g["n_rejected"][sl] == o["n_rejected"])
    np.testing.assert_array_equal(g["status"][sl], o["status"])
    e = rel_err(g["y_final"][:, sl], o["y_final"])[:, same]
    assert e.size == 0 or e.max() <= TOL, e.max()
    if "y_out" in o:
        e = rel_err(g["y_out"][:, :, sl], o["y_out"])[:, :, same]
        assert e.size == 0 or np.nanmax(e) <= TOL, np.nanmax(e)


def test_orbits_forward_full_config(orc):
    """1,000 orbits, Dopri5 1e-8/1e-10, 64 outputs: every output and count."""
    w = inputs.orbits_forward()
    g = to_np(gpu_solve(w))
    o = oracle_solve(orc, w)
    assert np.all(g["status"] == 0)
    _check(g, o)


CASES = [
    ("harmonic", lambda n: dict(rhs="harmonic", y0=np.random.default_rng(1).normal(size=(2, n)),
                                theta=np.random.default_rng(2).uniform(0.5, 2.0, (1, n)),
                                t0=0.0, t1=20.0, rtol=1e-9, atol=1e-9,
                                t_out=np.linspace(0.5, 20.0, 9))),
    ("kepler", lambda n: _kepler(n)),
    ("loghalo", lambda n: {**inputs.orbits_forward(n, seed=41), "t1": 30.0,
                           "t_out": np.linspace(0.0, 30.0, 13)}),
    ("spinprec", lambda n: {**inputs.spin_precession(n, seed=42), "t0": 100 ** -0.5,
                            "t_out": np.linspace(100 ** -0.5, 10 ** -0.5, 7)[1:]}),
    ("quint", lambda n: inputs.quintessence(n, seed=43)),
]


def _kepler(n):
    rng = np.random.default_rng(44)
    e = rng.uniform(0.0, 0.7, n)
    y0 = np.stack([1 - e, np.zeros(n), np.zeros(n), np.sqrt((1 + e) / (1 - e))])
    return dict(rhs="kepler", y0=y0, theta=np.array([1.0]), t0=0.0, t1=15.0, rtol=1e-10,
                atol=1e-10, t_out=np.linspace(1.0, 15.0, 8))


@pytest.mark.parametrize("tab", ["dopri5", "tsit5", "verner7"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_every_rhs_and_tableau(orc, name, make, tab):
    w = make(333)  # several waves and a ragged last one
    w["tableau"] = tab
    g = to_np(gpu_solve(w))
    o = oracle_solve(orc, w)
    assert np.all(g["status"] == 0)
    _check(g, o)


def test_uneven_batch_full_size_sampled(orc):
    """The full 100,000-orbit uneven batch on the GPU (persistent queue,
    longest-first order), in the benchmark's launch shapes with the head of
    the order on 16-lane groups: bitwise equal to one lane per trajectory,
    and 1,500 sampled orbits plus the 60 predicted-longest (on groups)
    recomputed by the oracle."""
    w = inputs.orbits_uneven()
    order = np.argsort(-inputs.predicted_cost(w), kind="stable")
    g = to_np(gpu_solve(w, order=order))
    assert np.all(g["status"] == 0)
    for L in (api.Launch(block=128, refill=8, wide=256),
              api.Launch(block=256, refill=4, wide=512)):
        gw = to_np(gpu_solve(w, L, order=order))
        for k in g:
            np.testing.assert_array_equal(gw[k], g[k], err_msg=f"{k} {L}")
    rnd = np.random.default_rng(7).choice(w["y0"].shape[1], 1500, replace=False)
    idx = np.unique(np.concatenate([rnd, order[:60]]))
    o = oracle_solve(orc, w, idx)
    _check(g, o, idx)


def test_schedules_and_shapes_are_bitwise_identical():
    """A trajectory's result does not depend on the lane it runs on."""
    w = inputs.orbits_uneven(n=3000, seed=45)
    ref = to_np(gpu_solve(w, api.Launch(schedule="static", block=64)))
    for L in (api.Launch(schedule="queue", block=256, refill=1),
              api.Launch(schedule="queue", block=128, refill=32, grid=7),
              api.Launch(schedule="queue", block=64, refill=64)):
        g = to_np(gpu_solve(w, L, order=np.random.default_rng(3).permutation(3000)))
        for k in ref:
            np.testing.assert_array_equal(g[k], ref[k])


def test_graph_replay_matches_direct_launch():
    w = inputs.orbits_forward(n=700, seed=46)
    direct = to_np(gpu_solve(w))
    prob = api.make_problem(w["rhs"], w["tableau"], w["y0"], w["theta"], w["t0"], w["t1"],
                            w["rtol"], w["atol"], w["t_out"])
    sol = api.Solution(prob, api.Launch())
    graph = api.Graph(sol)
    for _ in range(3):
        sol.y_final.fill_(0.0)
        sol.y_out.fill_(0.0)
        graph.launch()
        torch.cuda.synchronize()
        g = to_np(sol)
        for k in direct:
            np.testing.assert_array_equal(g[k], direct[k])
    graph.close()


def test_edge_cases(orc):
    w = inputs.orbits_forward(n=130, seed=47)
    y0 = w["y0"].copy()
    y0[1, 5] = np.nan
    t1 = np.full(130, 40.0)
    t1[7] = 0.0                      # empty span
    rtol = np.full(130, 1e-8)
    rtol[9] = -1.0                   # invalid tolerance
    w2 = {**w, "y0": y0, "t1": t1, "rtol": rtol, "atol": np.full(130, 1e-10),
          "t_out": np.array([0.0, 0.0, 0.0])}
    g = to_np(gpu_solve(w2, api.Launch(max_steps=0)))
    assert g["status"][5] == 3 and g["n_accepted"][5] == 0
    assert g["status"][7] == 0 and g["n_accepted"][7] == 0
    np.testing.assert_array_equal(g["y_final"][:, 7], y0[:, 7])
    assert g["status"][9] == 5 and np.all(np.isnan(g["y_out"][:, :, 9]))
    ok = [i for i in range(130) if i not in (5, 7, 9)]
    assert np.all(g["status"][ok] == 0)
    # max_steps
    g = to_np(gpu_solve(w, api.Launch(max_steps=25)))
    o = oracle_solve(orc, w, max_steps=25)
    np.testing.assert_array_equal(g["status"], o["status"])
    np.testing.assert_array_equal(g["n_accepted"] + g["n_rejected"],
                                  o["n_accepted"] + o["n_rejected"])


def test_empty_ensemble():
    w = inputs.orbits_forward(n=1, seed=48)
    prob = api.make_problem(w["rhs"], w["tableau"], np.zeros((6, 0)), w["theta"], 0.0, 1.0,
                            1e-8, 1e-10)
    api.solve(prob)
    torch.cuda.synchronize()


def test_rhs_vjp_matches_oracle_jacobian(orc):
    """Hand-written transposes J_y^T kbar, J_theta^T kbar on the GPU equal the
    oracle's forward-mode Jacobian applied by hand."""
    rng = np.random.default_rng(5)
    for name, make in CASES:
        w = make(64)
        d = w["y0"].shape[0]
        th = np.asarray(w["theta"], float)
        th = th if th.ndim == 2 else np.repeat(th[:, None], 64, axis=1)
        th = th[:, :64] if th.shape[1] >= 64 else np.repeat(th[:, :1], 64, axis=1)
        p = th.shape[0]
        y = w["y0"][:, :64] + 0.05 * rng.normal(size=(d, 64))
        t0 = float(np.asarray(w["t0"]).reshape(-1)[0])
        t1v = float(np.asarray(w["t1"]).reshape(-1)[0])
        t = rng.uniform(t0, t1v, 64)
        kb = rng.normal(size=(d, 64))
        f, yb, tb = api.rhs_eval(name, t, y, th, kb)
        f, yb, tb = f.cpu().numpy(), yb.cpu().numpy(), tb.cpu().numpy()
        for i in range(64):
            fo, J = orc.rhs(name, t[i], y[:, i], th[:, i], list(range(d + p)))
            np.testing.assert_allclose(f[:, i], fo, rtol=1e-13, atol=1e-13 * np.abs(fo).max())
            vj = kb[:, i] @ J
            scale = np.abs(vj).max() + 1e-300
            np.testing.assert_allclose(yb[:, i], vj[:d], rtol=0, atol=1e-12 * scale,
                                       err_msg=f"{name} ybar")
            np.testing.assert_allclose(tb[:, i], vj[d:], rtol=0, atol=1e-12 * scale,
                                       err_msg=f"{name} thetabar")


@pytest.mark.parametrize("tab", ["dopri5", "tsit5", "verner7"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_wide_groups_are_bitwise_identical(name, make, tab):
    """Trajectories run on 16-lane groups (one component per lane) take the
    same steps and give the same bits as on one lane, for every right-hand
    side and tableau; some of the ensemble on groups, or all of it."""
    w = {**make(333), "tableau": tab, "t_out": None}
    ref = to_np(gpu_solve(w))
    assert np.all(ref["status"] == 0)
    for wide in (37, 333):
        g = to_np(gpu_solve(w, api.Launch(wide=wide)))
        for k in ref:
            np.testing.assert_array_equal(g[k], ref[k], err_msg=f"{k} wide={wide}")


@pytest.mark.parametrize("tab", ["dopri5", "tsit5", "verner7"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_wide_groups_with_output_nodes(name, make, tab):
    """Groups with output nodes: the outputs (dense values, exact hits, nodes
    at t0 and t1, and for Verner 7 the deferred shortened steps), final
    states and counts are bitwise those of one lane per trajectory, in both
    output layouts."""
    w = {**make(333), "tableau": tab}
    for layout in ("dkn", "knd"):
        ref = to_np(gpu_solve(w, api.Launch(out_layout=layout)))
        assert np.all(ref["status"] == 0)
        for wide in (37, 333):
            g = to_np(gpu_solve(w, api.Launch(wide=wide, out_layout=layout)))
            for k in ref:
                np.testing.assert_array_equal(g[k], ref[k], err_msg=f"{k} wide={wide} {layout}")


@pytest.mark.parametrize("tab", ["dopri5", "verner7"])
def test_wide_group_outputs_of_stopped_and_invalid_trajectories(tab):
    """Per-trajectory output times; a trajectory with a non-finite state, one
    with an empty span and trajectories stopped by the step limit: the NaN
    outputs past where each stopped, bitwise those of one lane each."""
    n = 300
    w = {**inputs.orbits_forward(n, seed=53), "tableau": tab}
    tk = np.sort(np.random.default_rng(54).uniform(0.0, 50.0, (24, n)), axis=0)
    tk[0, :] = 0.0                                   # a node at t0
    y0 = w["y0"].copy()
    y0[2, 5] = np.nan
    t1 = np.full(n, float(np.max(w["t1"])))
    t1[9] = float(np.min(w["t0"]))                   # empty span
    w = {**w, "y0": y0, "t1": t1, "t_out": tk}
    for L in (dict(), dict(max_steps=300)):
        ref = to_np(gpu_solve(w, api.Launch(**L)))
        g = to_np(gpu_solve(w, api.Launch(wide=n, **L)))
        assert ref["status"][5] != 0
        if L:
            assert np.any(ref["status"] != 0) and np.any(np.isnan(ref["y_out"][:, -1, :]))
        for k in ref:
            np.testing.assert_array_equal(g[k], ref[k], err_msg=f"{k} {L}")


def test_wide_groups_on_the_uneven_batch(orc):
    """Longest-first order with the 300 predicted-longest orbits of 20,000 on
    groups: bitwise equal to one lane each, and to the oracle on a sample."""
    w = inputs.orbits_uneven(n=20_000, seed=47)
    order = np.argsort(-inputs.predicted_cost(w), kind="stable")
    ref = to_np(gpu_solve(w, order=order))
    g = to_np(gpu_solve(w, api.Launch(wide=300, block=128), order=order))
    for k in ref:
        np.testing.assert_array_equal(g[k], ref[k])
    idx = np.sort(np.concatenate([order[:60], order[-40:]]))
    _check(g, oracle_solve(orc, w, idx), idx)


@pytest.mark.parametrize("grid,wide", [(3, 500), (2, 2000), (6, 40)], ids=["g3w500", "g2wall", "g6w40"])
def test_wide_groups_with_a_small_grid(grid, wide):
    """More wide trajectories than groups the grid holds: the groups refill
    from their own queue, at least one workgroup keeps the single lanes, and
    the results are bitwise those of one lane per trajectory."""
    w = inputs.orbits_uneven(n=2000, seed=48)
    w = {**w, "t1": np.minimum(w["t1"], 40.0)}
    order = np.argsort(-inputs.predicted_cost(w), kind="stable")
    ref = to_np(gpu_solve(w, order=order))
    g = to_np(gpu_solve(w, api.Launch(block=64, grid=grid, wide=wide), order=order))
    assert np.all(ref["status"] == 0)
    for k in ref:
        np.testing.assert_array_equal(g[k], ref[k], err_msg=k)


@pytest.mark.parametrize("tab", ["dopri5", "tsit5", "verner7"])
def test_output_layout_knd(tab):
    """y_out in [K][n][d] holds the default [d][K][n] outputs transposed, bit
    for bit, for polynomial and shortened-step outputs, shared and
    per-trajectory output times, and the NaN outputs of trajectories stopped
    before them."""
    w = {**inputs.orbits_forward(300, seed=50), "tableau": tab}
    tk = np.sort(np.random.default_rng(51).uniform(0.0, 50.0, (24, 300)), axis=0)
    for wt in (w, {**w, "t_out": tk}):
        for L0, L1 in ((api.Launch(), api.Launch(out_layout="knd")),
                       (api.Launch(max_steps=300), api.Launch(max_steps=300, out_layout="knd"))):
            a = to_np(gpu_solve(wt, L0))
            b = to_np(gpu_solve(wt, L1))
            np.testing.assert_array_equal(b["y_out"], a["y_out"].transpose(1, 2, 0))
            for k in ("y_final", "n_accepted", "n_rejected", "status"):
                np.testing.assert_array_equal(b[k], a[k], err_msg=k)


@pytest.mark.parametrize("tab", ["dopri5", "verner7"])
def test_wide_groups_write_the_checkpoint_tape(tab):
    """Groups with a checkpoint-mode tape (every 5 accepted steps, PI control
    so that the controller memory is on it too): the tape bytes and results
    of one lane per trajectory, the adjoint's replay lands on every next
    checkpoint, and the gradients are the same; with a tape too short, the
    same overflow status."""
    n = 2000
    w = inputs.orbits_uneven(n=n, seed=55)
    w = {**w, "t1": np.minimum(w["t1"], 40.0), "tableau": tab}
    order = np.argsort(-inputs.predicted_cost(w), kind="stable")
    p = api.make_problem(w["rhs"], tab, w["y0"], w["theta"], w["t0"], w["t1"], w["rtol"],
                         w["atol"])
    ctl = dict(beta1=0.7 / 5, beta2=0.4 / 5) if tab == "dopri5" else {}
    nmax = int(api.solve(p, api.Launch(**ctl)).n_accepted.max())
    for cap in (nmax // 5 + 2, 5):
        sols = []
        for wide in (0, 400):
            s = api.Solution(p, api.Launch(block=128, ckpt_every=5, ckpt_capacity=cap, wide=wide,
                                           **ctl))
            s.set_order(order)
            s.workspace.zero_()
            s.run()
            sols.append(s)
        torch.cuda.synchronize()
        a, b = sols
        for k in ("y_final", "n_accepted", "n_rejected", "status"):
            assert torch.equal(getattr(a, k), getattr(b, k)), k
        tape_bytes = n * cap * (3 + 2 * 6) * 8
        assert torch.equal(a.workspace[256:256 + tape_bytes], b.workspace[256:256 + tape_bytes])
        if cap == 5:
            assert bool((a.status == 4).any())
            continue
        assert bool((a.status == 0).all())
        yb = torch.ones((1, 6, n), dtype=torch.float64, device="cuda")
        ga = api.solve_vjp(a, ybar_final=yb)
        gb = api.solve_vjp(b, ybar_final=yb)
        torch.cuda.synchronize()
        assert a.replay_mismatches() == 0 and b.replay_mismatches() == 0
        for x, y in zip(ga, gb):
            assert torch.equal(x, y)


@pytest.mark.parametrize("k", [1, 4], ids=["store", "ckpt4"])
def test_wide_groups_with_outputs_and_a_tape(k):
    """Groups writing output nodes (deferred records) and a tape in the same
    launch: outputs, tape bytes and gradients with output cotangents are
    those of one lane per trajectory."""
    n = 600
    w = inputs.orbits_forward(n=n, seed=56)
    w = {**w, "t_out": w["t_out"][::4]}
    order = np.random.default_rng(57).permutation(n)
    p = api.make_problem(w["rhs"], w["tableau"], w["y0"], w["theta"], w["t0"], w["t1"],
                         w["rtol"], w["atol"], w["t_out"])
    nmax = int(api.solve(p).n_accepted.max())
    cap = nmax // k + 2
    sols = []
    for wide in (0, 200):
        s = api.Solution(p, api.Launch(block=128, ckpt_every=k, ckpt_capacity=cap, wide=wide))
        s.set_order(order)
        s.workspace.zero_()
        s.run()
        sols.append(s)
    torch.cuda.synchronize()
    a, b = sols
    for key in ("y_final", "y_out", "n_accepted", "n_rejected", "status"):
        assert torch.equal(getattr(a, key), getattr(b, key)), key
    rec = 2 + 6 if k == 1 else 3 + 2 * 6
    tape_bytes = n * cap * rec * 8
    assert torch.equal(a.workspace[256:256 + tape_bytes], b.workspace[256:256 + tape_bytes])
    yo = torch.as_tensor(np.random.default_rng(58).normal(size=(1, 6, p.K, n)), device="cuda")
    yf = torch.ones((1, 6, n), dtype=torch.float64, device="cuda")
    ga = api.solve_vjp(a, ybar_final=yf, ybar_out=yo)
    gb = api.solve_vjp(b, ybar_final=yf, ybar_out=yo)
    torch.cuda.synchronize()
    for x, y in zip(ga, gb):
        assert torch.equal(x, y)
    assert bool(torch.isfinite(ga[0]).all())


def test_wide_groups_write_the_store_tape():
    """Groups with a store-mode tape: the tape bytes, results and statuses of
    one lane per trajectory, and the same adjoint gradients from it; with a
    tape too short, the same overflow status."""
    w = inputs.orbits_uneven(n=3000, seed=52)
    w = {**w, "t1": np.minimum(w["t1"], 60.0)}
    order = np.argsort(-inputs.predicted_cost(w), kind="stable")
    p = api.make_problem(w["rhs"], w["tableau"], w["y0"], w["theta"], w["t0"], w["t1"],
                         w["rtol"], w["atol"])
    nmax = int(api.solve(p).n_accepted.max())
    for cap in (nmax + 2, 40):
        sols = []
        for wide in (0, 500):
            s = api.Solution(p, api.Launch(block=128, ckpt_every=1, ckpt_capacity=cap, wide=wide))
            s.set_order(order)
            s.workspace.zero_()  # records past a trajectory's last step are never written
            s.run()
            sols.append(s)
        torch.cuda.synchronize()
        a, b = sols
        for k in ("y_final", "n_accepted", "n_rejected", "status"):
            assert torch.equal(getattr(a, k), getattr(b, k)), k
        tape_bytes = 3000 * cap * (2 + 6) * 8
        assert torch.equal(a.workspace[256:256 + tape_bytes], b.workspace[256:256 + tape_bytes])
        if cap == 40:
            assert bool((a.status == 4).any())
            continue
        assert bool((a.status == 0).all())
        yb = torch.ones((1, 6, 3000), dtype=torch.float64, device="cuda")
        ga = api.solve_vjp(a, ybar_final=yb)
        gb = api.solve_vjp(b, ybar_final=yb)
        for x, y in zip(ga, gb):
            assert torch.equal(x, y)
