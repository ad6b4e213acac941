"""The benchmark configurations at full size on the GPU: parity with the
oracle on sampled trajectories, and the paper's accuracy budgets against the
oracle's tight reference (Section "How the codes are compared", eq:accept;
Appendix "References, tolerances and timing").

Budgets: orbits 1e-4 of the orbit's own size and speed (eq:st-fwderr);
dark-energy distances 1e-4 c/H0; precession angles 2e-7 rad (eq:prec-err).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import oracle_solve, rel_err, to_np  # noqa: E402
from parity_log import record  # noqa: E402
from paper_2609_28458_amd import api, inputs  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    api.lib()


def _prob(w, idx=None, **over):
    w = {**w, **over}
    return api.make_problem(w["rhs"], w["tableau"], w["y0"], w["theta"], w["t0"], w["t1"],
                            w["rtol"], w["atol"], w.get("t_out"))


def _parity(g, o, idx, what="config"):
    np.testing.assert_array_equal(g["n_accepted"][idx], o["n_accepted"])
    np.testing.assert_array_equal(g["n_rejected"][idx], o["n_rejected"])
    e = np.max(rel_err(g["y_final"][:, idx], o["y_final"]))
    if "y_out" in o:
        e = max(e, np.max(rel_err(g["y_out"][:, :, idx], o["y_out"])))
    record(what, e, 1e-9)
    assert e <= 1e-9, e


def _p99(x):
    return float(np.quantile(x, 0.99))


def test_orbits_forward_budget(orc):
    """1,000 orbits: P99 of eps^y over the outputs against Verner 7 at 1e-13
    within 1e-4 of each orbit's r_E, v_E (eq:st-scales, eq:st-fwderr)."""
    w = inputs.orbits_forward()
    g = to_np(api.solve(_prob(w)))
    ref = orc.solve(w["rhs"], "verner7", w["y0"], w["theta"], 0.0, 50.0, 1e-13, 1e-13,
                    w["t_out"])
    v0, q, rc = w["theta"]
    y = w["y0"]
    Dn = rc * rc + y[0] ** 2 + y[1] ** 2 + y[2] ** 2 / q ** 2
    E = 0.5 * (y[3] ** 2 + y[4] ** 2 + y[5] ** 2) + 0.5 * v0 * v0 * np.log(Dn)
    rE = np.sqrt(np.exp(2 * E / v0 ** 2) - rc * rc)        # Phi(r_E, 0) = E
    vE = np.sqrt(2 * E - v0 * v0 * np.log(rc * rc))         # v_E^2/2 + Phi(0, 0) = E
    dx = np.linalg.norm(g["y_out"][:3] - ref["y_out"][:3], axis=0) / rE
    dv = np.linalg.norm(g["y_out"][3:] - ref["y_out"][3:], axis=0) / vE
    eps = np.maximum(dx, dv).max(axis=0)
    assert np.all(np.isfinite(eps)) and _p99(eps) <= 1e-4, _p99(eps)


def _orbit_scales(y, v0, q, rc):
    """r_E and v_E of each orbit (eq:st-scales) from its energy."""
    Dn = rc * rc + y[0] ** 2 + y[1] ** 2 + y[2] ** 2 / q ** 2
    E = 0.5 * (y[3] ** 2 + y[4] ** 2 + y[5] ** 2) + 0.5 * v0 * v0 * np.log(Dn)
    return np.sqrt(np.exp(2 * E / v0 ** 2) - rc * rc), np.sqrt(2 * E - v0 * v0 * np.log(rc * rc))


def test_streams_within_the_paper_budgets(orc):
    """The paper's stream workload (10^4 orbits of inputs.streams, Tsit5 at
    3.16e-7): the final state and its sensitivity to (v_c, q), taken in the
    same launch, against Verner 7 at 1e-12 with sensitivities.  The 99th
    percentiles of eps^y (eq:st-fwderr) and eps^S (eq:st-graderr: rows
    scaled by 1/r_E and 1/v_E, columns by v_c and q, Frobenius norms) must
    meet the paper's budgets, 1e-4 and 1e-3 (eq:accept)."""
    w = inputs.streams(n=10_000, seed=19)
    prob = _prob(w)
    g = to_np(api.solve(prob))
    _, S, _ = api.solve_sens(prob, w["grad_cols"])
    torch.cuda.synchronize()
    S = S.cpu().numpy()                                     # [6][2][n]
    ref = orc.solve(w["rhs"], "verner7", w["y0"], w["theta"], 0.0, w["t1"], 1e-12, 1e-12,
                    sens_cols=w["grad_cols"])
    v0, q, rc = w["theta"]
    rE, vE = _orbit_scales(w["y0"], v0, q, rc)
    dx = np.linalg.norm(g["y_final"][:3] - ref["y_final"][:3], axis=0) / rE
    dv = np.linalg.norm(g["y_final"][3:] - ref["y_final"][3:], axis=0) / vE
    eps_y = np.maximum(dx, dv)
    Wrow = np.concatenate([np.broadcast_to(1 / rE, (3, rE.size)),
                           np.broadcast_to(1 / vE, (3, vE.size))])[:, None, :]
    Dcol = np.array([v0, q])[None, :, None]
    num = np.linalg.norm((Wrow * (S - ref["S_final"]) * Dcol).reshape(12, -1), axis=0)
    den = np.linalg.norm((Wrow * ref["S_final"] * Dcol).reshape(12, -1), axis=0)
    eps_s = num / den
    print(f"streams P99: eps_y {_p99(eps_y):.2e} (paper 5.7e-5), eps_S {_p99(eps_s):.2e} "
          f"(paper 6e-4); mean attempts {(g['n_accepted'] + g['n_rejected']).mean():.1f}")
    assert np.all(g["status"] == 0)
    assert _p99(eps_y) <= 1e-4 and _p99(eps_s) <= 1e-3


def _angle_error(a, b):
    """eq:prec-err: the largest angle between the final L, S1, S2 of two runs."""
    eps = np.zeros(a.shape[1])
    for s in range(3):
        x, y = a[3 * s:3 * s + 3], b[3 * s:3 * s + 3]
        ang = np.arctan2(np.linalg.norm(np.cross(x, y, axis=0), axis=0), np.sum(x * y, axis=0))
        eps = np.maximum(eps, ang)
    return eps


def test_spin_precession_full_size(orc):
    """10^6 binaries from r = 1000 to 10 with Verner 7 at 3.16e-9 and 32
    outputs: parity on 1,000 sampled binaries plus the 50 that took the most
    attempts.  From r = 1000 this tolerance does not meet the 2e-7 rad
    budget (about 30 times more precession cycles than from r = 100); the
    error is printed, and the budget is checked at the loosest passing
    tolerance below."""
    w = inputs.spin_precession()
    n = w["y0"].shape[1]
    g = to_np(api.solve(_prob(w)))
    assert np.all(g["status"] == 0)
    longest = np.argsort(-(g["n_accepted"] + g["n_rejected"]))[:50]
    idx = np.unique(np.concatenate([np.random.default_rng(9).choice(n, 1000, replace=False),
                                    longest]))
    o = oracle_solve(orc, w, idx)
    np.testing.assert_array_equal(g["n_accepted"][idx], o["n_accepted"])
    np.testing.assert_array_equal(g["n_rejected"][idx], o["n_rejected"])
    # Over up to ~88,000 steps the precession amplifies rounding: changing the
    # parameters by two ulps moves the oracle's own final directions by up to
    # 1.4e-9 at identical step counts.  The GPU evaluates the right-hand side
    # with fused multiply-adds where the oracle rounds every product, a
    # difference of a few ulps per evaluation.  A single perturbation's
    # effect on one binary is itself a draw (it can happen to be small), so
    # each binary's sensitivity is the largest effect of three perturbations
    # of that size (the parameters by -1e-15, +1e-15 and +4e-16 relative),
    # and its bar is 1e-9 or five times that, whichever is larger.
    self_d = np.zeros(len(idx))
    for rel in (-1e-15, 1e-15, 4e-16):
        th2 = w["theta"][:, idx] * (1.0 + rel)
        o2 = orc.solve(w["rhs"], w["tableau"], w["y0"][:, idx], th2, w["t0"], w["t1"],
                       w["rtol"], w["atol"], w["t_out"])
        self_d = np.maximum(self_d, np.maximum(
            np.abs(o2["y_final"] - o["y_final"]).max(axis=0),
            np.abs(o2["y_out"] - o["y_out"]).max(axis=(0, 1))))
    bar = np.maximum(1e-9, 5.0 * self_d)
    e = np.maximum(rel_err(g["y_final"][:, idx], o["y_final"]).max(axis=0),
                   rel_err(g["y_out"][:, :, idx], o["y_out"]).max(axis=(0, 1)))
    record("precession 10^6 at 3.16e-9, 1,050 sampled incl. the 50 longest: max error "
           "(bar: that binary's own)", e.max(), bar[np.argmax(e)])
    record("  same, error over the binary's own bar (<= 1)", (e / bar).max(), 1.0)
    record("  same, binaries whose own rounding response exceeds 2e-10", (self_d > 2e-10).sum(),
           len(idx))
    assert np.all(e <= bar), (e.max(), (e / bar).max())
    idx = idx[:100]
    o = {k: v[..., :100] for k, v in o.items()}
    ref = orc.solve("spinprec", "verner7", w["y0"][:, idx], w["theta"][:, idx], w["t0"], w["t1"],
                    1e-13, 1e-13)
    eps = _angle_error(g["y_final"][:, idx], ref["y_final"])
    print(f"precession from r=1000 at 3.16e-9: P99 angle error {_p99(eps):.3e} rad on 100 "
          f"binaries; mean attempts {np.mean(g['n_accepted'] + g['n_rejected']):.0f}")
    assert np.all(np.isfinite(eps))


def test_spin_precession_headline_configuration(orc):
    """The benchmark's headline as it is timed: 10^6 binaries from r = 1000
    at 1e-11 with 32 outputs, longest first by the device order of a
    pilot-fitted cost, refill at one idle lane.  Parity on 400 sampled
    binaries plus the 20 that took the most attempts, each within 1e-9 or
    five times the oracle's own response to rounding-level parameter
    changes (the largest of three), with identical step counts."""
    from paper_2609_28458_amd import autotune

    w = inputs.spin_precession()
    w.update(rtol=1e-11, atol=1e-11)
    n = w["y0"].shape[1]
    prob = _prob(w)
    pilot = _prob({**w, "t0": 100.0 ** -0.5, "t_out": None})
    y, th = pilot.y0, pilot.theta
    feats = torch.stack([torch.log(th[0]), th[1], th[2], (y[0:3] * y[3:6]).sum(0),
                         (y[0:3] * y[6:9]).sum(0), (y[3:6] * y[6:9]).sum(0)])
    cost = autotune.pilot_cost(pilot, feats).contiguous()
    sol = api.Solution(prob, api.Launch(refill=1))
    sol.queue_order(cost)
    sol.run()
    torch.cuda.synchronize()
    g = to_np(sol)
    assert np.all(g["status"] == 0)
    longest = np.argsort(-(g["n_accepted"] + g["n_rejected"]))[:20]
    idx = np.unique(np.concatenate([np.random.default_rng(14).choice(n, 400, replace=False),
                                    longest]))
    o = oracle_solve(orc, w, idx)
    np.testing.assert_array_equal(g["n_accepted"][idx], o["n_accepted"])
    np.testing.assert_array_equal(g["n_rejected"][idx], o["n_rejected"])
    self_d = np.zeros(len(idx))
    for rel in (-1e-15, 1e-15, 4e-16):
        o2 = orc.solve(w["rhs"], w["tableau"], w["y0"][:, idx], w["theta"][:, idx] * (1.0 + rel),
                       w["t0"], w["t1"], w["rtol"], w["atol"], w["t_out"])
        self_d = np.maximum(self_d, np.maximum(
            np.abs(o2["y_final"] - o["y_final"]).max(axis=0),
            np.abs(o2["y_out"] - o["y_out"]).max(axis=(0, 1))))
    bar = np.maximum(1e-9, 5.0 * self_d)
    e = np.maximum(rel_err(g["y_final"][:, idx], o["y_final"]).max(axis=0),
                   rel_err(g["y_out"][:, :, idx], o["y_out"]).max(axis=(0, 1)))
    record("precession headline (10^6 at 1e-11, device order, refill 1), 420 sampled incl. "
           "the 20 longest: max error (bar: that binary's own)", e.max(), bar[np.argmax(e)])
    record("  same, error over the binary's own bar (<= 1)", (e / bar).max(), 1.0)
    assert np.all(e <= bar), (e.max(), (e / bar).max())


def test_spin_precession_paper_setting(orc):
    """The paper's own setting, r = 100 M to 10 M, 10^6 binaries, Verner 7 at
    3.16e-9: mean attempts over the whole population near its 911, and the
    99th percentile of eq:prec-err within 2e-7 rad on 300 sampled binaries
    (parity on the same sample)."""
    w = inputs.spin_precession()
    w["t0"] = 100.0 ** -0.5
    w["t_out"] = None
    n = w["y0"].shape[1]
    g = to_np(api.solve(_prob(w)))
    assert np.all(g["status"] == 0)
    att = np.mean(g["n_accepted"] + g["n_rejected"])
    assert abs(att / 911 - 1) < 0.02, att
    idx = np.sort(np.random.default_rng(11).choice(n, 300, replace=False))
    _parity(g, oracle_solve(orc, w, idx), idx)
    ref = orc.solve("spinprec", "verner7", w["y0"][:, idx], w["theta"][:, idx], w["t0"], w["t1"],
                    1e-13, 1e-13)
    eps = _angle_error(g["y_final"][:, idx], ref["y_final"])
    print(f"precession from r=100: P99 {_p99(eps):.3e} rad, mean attempts {att:.1f}")
    assert _p99(eps) <= 2e-7


def test_spin_precession_budget_from_r1000(orc):
    """From r = 1000 the loosest tolerance on the quarter-decade grid that
    meets the 2e-7 rad budget is 1e-11 (Verner 7): checked on 200 binaries of
    a 20,000-binary GPU run."""
    w = inputs.spin_precession(n=20_000, seed=12)
    w.update(rtol=1e-11, atol=1e-11, t_out=None)
    g = to_np(api.solve(_prob(w)))
    assert np.all(g["status"] == 0)
    idx = np.sort(np.random.default_rng(13).choice(20_000, 200, replace=False))
    ref = orc.solve("spinprec", "verner7", w["y0"][:, idx], w["theta"][:, idx], w["t0"], w["t1"],
                    1e-14, 1e-14)
    eps = _angle_error(g["y_final"][:, idx], ref["y_final"])
    print(f"precession from r=1000 at 1e-11: P99 {_p99(eps):.3e} rad, mean attempts "
          f"{np.mean(g['n_accepted'] + g['n_rejected']):.0f}")
    assert _p99(eps) <= 2e-7


def test_spin_precession_tilt_gradients(orc):
    """Gradients of both final tilt angles with respect to (q, chi1, chi2)
    for the 20,000-binary subset (two losses share one adjoint replay),
    checked against the oracle's forward sensitivities on 40 binaries."""
    w = inputs.spin_precession(n=20_000)
    n = 20_000
    plain = api.solve(_prob(w, t_out=None))
    torch.cuda.synchronize()
    k = 128
    cap = int(plain.n_accepted.max()) // k + 2
    sol = api.solve(_prob(w, t_out=None), api.Launch(ckpt_every=k, ckpt_capacity=cap))
    torch.cuda.synchronize()
    assert bool((sol.status == 0).all())
    y = sol.y_final.detach().clone().requires_grad_(True)
    L, S1, S2 = y[:3], y[3:6], y[6:9]

    def tilt(a, b):
        return torch.atan2(torch.linalg.norm(torch.cross(a, b, dim=0), dim=0), (a * b).sum(0))

    ybar = torch.zeros((2, 9, n), dtype=torch.float64, device="cuda")
    for r, S in enumerate((S1, S2)):
        (gr,) = torch.autograd.grad(tilt(L, S).sum(), y)
        ybar[r] = gr
    y0b, thb = api.solve_vjp(sol, ybar_final=ybar)
    torch.cuda.synchronize()
    assert sol.replay_mismatches() == 0
    idx = np.sort(np.random.default_rng(10).choice(n, 40, replace=False))
    o = oracle_solve(orc, w, idx, sens_cols=[9, 10, 11])
    yb = ybar.cpu().numpy()[:, :, idx]
    ref = np.einsum("rjn,jcn->rcn", yb, o["S_final"])
    got = thb.cpu().numpy()[:, :, idx]
    scale = np.maximum(np.abs(ref).max(axis=1, keepdims=True), 1e-6)
    err = np.max(np.abs(got - ref) / scale)
    # the gradient's own response to rounding-level changes of the parameters
    # (the same amplification of rounding as for the solution; the largest of
    # three draws)
    self_d = 0.0
    for rel in (-1e-15, 1e-15, 4e-16):
        o2 = oracle_solve(orc, {**w, "theta": w["theta"] * (1.0 + rel)}, idx,
                          sens_cols=[9, 10, 11])
        ref2 = np.einsum("rjn,jcn->rcn", yb, o2["S_final"])
        self_d = max(self_d, np.max(np.abs(ref2 - ref) / scale))
    bar = max(1e-7, 5.0 * self_d)
    record("tilt-angle gradients vs oracle FS (40 binaries from r = 1000; bar max(1e-7, 5 x "
           f"the oracle's response to rounding, {self_d:.2g}))", err, bar)
    assert err < bar


@pytest.mark.parametrize("dense", [False, True])
def test_quintessence_full_size(orc, dense):
    """10^4 cosmologies, Dopri5 at 1.78e-4 / 1.78e-7, distances at 7 (dense
    variant 64) redshifts: parity on every cosmology, and the distance error
    max(|dD_M|, |dD_H|) in units of c/H0 against the tight reference (Verner
    7 at 1e-11 / 1e-13) within 1e-4 at the 99th percentile."""
    w = inputs.quintessence(dense=dense)
    n = w["y0"].shape[1]
    g = to_np(api.solve(_prob(w)))
    assert np.all(g["status"] == 0)
    o = oracle_solve(orc, w)
    _parity(g, o, np.arange(n))
    ref = orc.solve("quint", "verner7", w["y0"], w["theta"], w["t0"], w["t1"], 1e-11, 1e-13,
                    w["t_out"])
    a0, lam, om, orad = w["theta"]
    N = w["t_out"][:, None]

    def dist(yo, yf):
        E = np.sqrt((om * np.exp(-3 * N) + orad * np.exp(-4 * N) + a0 * np.exp(-lam * yo[0]))
                    / (1 - yo[1] ** 2 / 6))
        return yf[2][None, :] - yo[2], 1.0 / E

    dm, dh = dist(g["y_out"], g["y_final"])
    rm, rh = dist(ref["y_out"], ref["y_final"])
    eps = np.maximum(np.abs(dm - rm), np.abs(dh - rh)).max(axis=0)
    print(f"dark-energy P99 distance error: {_p99(eps):.3e} c/H0 (budget 1e-4)")
    assert np.all(np.isfinite(eps)) and _p99(eps) <= 1e-4
