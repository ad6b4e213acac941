"""Pins of the oracle's adaptive loop (eq:rk, eq:errnorm, eq:controller,
eq:dense) against things fixed independently of it:

* scipy's RK45 is the Dormand--Prince 5(4) pair with the same RMS norm
  (eq:errnorm), the same starting-step rule and an I controller that differs
  from eq:controller only in its growth cap (10) and in not growing the step
  right after a rejection.  With those two settings the oracle must take
  exactly scipy's steps and agree to rounding, dense outputs included.
* Fixed-step global error on the harmonic oscillator scales as h^nu
  (nu = 5, 5, 7), dense outputs as h^4 or better.
* Controller branches: err = 0 grows by alpha_max, NaN fails the trajectory.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from paper_2609_28458_amd import inputs


def loghalo_np(theta):
    v0, q, rc = theta

    def f(t, y):
        D = rc * rc + y[0] ** 2 + y[1] ** 2 + y[2] ** 2 / q ** 2
        s = -v0 * v0 / D
        return np.array([y[3], y[4], y[5], s * y[0], s * y[1], s * y[2] / q ** 2])

    return f


def test_dopri5_equals_scipy_rk45(orc):
    w = inputs.orbits_forward(n=12, seed=11)
    o = orc.solve(w["rhs"], "dopri5", w["y0"], w["theta"], 0.0, 50.0, 1e-8, 1e-10,
                  w["t_out"], alpha_max=10.0, no_grow_after_reject=True)
    f = loghalo_np(w["theta"])
    for i in range(12):
        s = solve_ivp(f, (0.0, 50.0), w["y0"][:, i], method="RK45", rtol=1e-8, atol=1e-10,
                      t_eval=w["t_out"])
        attempts = (s.nfev - 2) // 6  # 2 calls for the starting step, 6 per attempt
        assert o["n_accepted"][i] + o["n_rejected"][i] == attempts
        np.testing.assert_allclose(o["y_final"][:, i], s.y[:, -1], rtol=0, atol=1e-11)
        np.testing.assert_allclose(o["y_out"][:, :, i], s.y, rtol=0, atol=1e-11)


def _fixed_steps(orc, tab, N, T=10.0, nodes=None):
    y0 = np.array([[1.0], [0.3]])
    hs = np.full((1, N), T / N)
    return orc.solve("harmonic", tab, y0, np.array([1.3]), 0.0, T, 1e-6, 1e-6, nodes,
                     h_replay=hs, n_replay=[N])


def _exact_harmonic(t, x0=1.0, v0=0.3, w=1.3):
    return x0 * np.cos(w * t) + v0 / w * np.sin(w * t)


@pytest.mark.parametrize("tab,nu,Ns", [("dopri5", 5, (40, 80, 160)),
                                       ("tsit5", 5, (40, 80, 160)),
                                       ("verner7", 7, (20, 40, 80))])
def test_fixed_step_convergence_order(orc, tab, nu, Ns):
    errs = []
    for N in Ns:
        o = _fixed_steps(orc, tab, N)
        assert o["n_accepted"][0] == N and o["status"][0] == 0
        errs.append(abs(o["y_final"][0, 0] - _exact_harmonic(10.0)))
    slopes = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert all(abs(s - nu) < 0.3 for s in slopes), (errs, slopes)


@pytest.mark.parametrize("tab,lo", [("dopri5", 3.7), ("tsit5", 3.7), ("verner7", 6.6)])
def test_dense_output_order(orc, tab, lo):
    """Outputs in the interior of steps converge at the interpolant's order."""
    T = 10.0
    nodes = np.array([1.234, 3.7001, 5.55, 7.9, 9.87])
    errs = []
    for N in (40, 80, 160):
        o = _fixed_steps(orc, tab, N, T, nodes)
        errs.append(np.max(np.abs(o["y_out"][0, :, 0] - _exact_harmonic(nodes))))
    slopes = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(slopes) > lo, (errs, slopes)


def test_dense_output_endpoints(orc):
    """A node at the end of an accepted step returns y+ itself; a node at t0
    returns y0; a node at t1 equals the final state."""
    w = inputs.orbits_forward(n=4, seed=12)
    rec = orc.solve(w["rhs"], "tsit5", w["y0"], w["theta"], 0.0, 5.0, 1e-8, 1e-10, h_cap=4000)
    h = rec["h_rec"][0, :rec["n_accepted"][0]]
    t_end3 = h[0] + h[1] + h[2]
    nodes = np.array([0.0, t_end3, 5.0])
    o = orc.solve(w["rhs"], "tsit5", w["y0"][:, :1], w["theta"], 0.0, 5.0, 1e-8, 1e-10, nodes)
    np.testing.assert_array_equal(o["y_out"][:, 0, 0], w["y0"][:, 0])
    np.testing.assert_array_equal(o["y_out"][:, 2, 0], o["y_final"][:, 0])
    # value at the end of step 3 from a replay of exactly three steps
    o3 = orc.solve(w["rhs"], "tsit5", w["y0"][:, :1], w["theta"], 0.0, t_end3, 1e-8, 1e-10,
                   h_replay=h[None, :3], n_replay=[3])
    np.testing.assert_array_equal(o["y_out"][:, 1, 0], o3["y_final"][:, 0])


def test_verner7_shortened_step_is_a_true_step(orc):
    """For Verner 7 an output at t + sigma h equals one step of length sigma h."""
    w = inputs.orbits_forward(n=1, seed=13)
    rec = orc.solve(w["rhs"], "verner7", w["y0"], w["theta"], 0.0, 3.0, 1e-9, 1e-9, h_cap=1000)
    h = rec["h_rec"][0]
    t2 = h[0] + h[1]
    tq = t2 + 0.37 * h[2]
    o = orc.solve(w["rhs"], "verner7", w["y0"], w["theta"], 0.0, 3.0, 1e-9, 1e-9, [tq])
    hs = np.array([[h[0], h[1], tq - t2]])
    o2 = orc.solve(w["rhs"], "verner7", w["y0"], w["theta"], 0.0, tq, 1e-9, 1e-9,
                   h_replay=hs, n_replay=[3])
    np.testing.assert_allclose(o["y_out"][:, 0, 0], o2["y_final"][:, 0], rtol=0, atol=1e-15)


def test_controller_zero_error_grows_by_alpha_max(orc):
    """f = 0 everywhere (oscillator at rest with omega = 0): every error is 0,
    so each accepted step grows by exactly alpha_max."""
    o = orc.solve("harmonic", "tsit5", np.zeros((2, 1)), np.array([0.0]), 0.0, 1e6, 1e-6, 1e-6,
                  h0=1e-3, h_cap=50)
    h = o["h_rec"][0, :o["n_accepted"][0]]
    assert o["n_rejected"][0] == 0 and o["status"][0] == 0
    np.testing.assert_array_equal(h[1:-1] / h[:-2], 5.0)


def test_controller_rejects_then_shrinks(orc):
    """A deliberately too-large first step is rejected, and the retry is
    shorter by the factor of eq:controller, clamped to [alpha_min, alpha_max]."""
    w = inputs.orbits_forward(n=1, seed=14)
    o = orc.solve(w["rhs"], "dopri5", w["y0"], w["theta"], 0.0, 50.0, 1e-10, 1e-10, h0=2.0,
                  h_cap=5000)
    assert o["n_rejected"][0] >= 1
    first = o["h_rec"][0, 0]
    assert first < 2.0 * 0.9 and first >= 2.0 * 0.2 ** o["n_rejected"][0] * 0.999


def test_failure_statuses(orc):
    w = inputs.orbits_forward(n=3, seed=15)
    y0 = w["y0"].copy()
    y0[0, 1] = np.nan
    o = orc.solve(w["rhs"], "dopri5", y0, w["theta"], 0.0, 50.0, 1e-8, 1e-10, w["t_out"],
                  max_steps=10)
    assert o["status"][0] == 1 and o["n_accepted"][0] + o["n_rejected"][0] == 10
    assert o["status"][1] == 3 and o["n_accepted"][1] + o["n_rejected"][1] == 0
    assert np.all(np.isnan(o["y_out"][:, -1, 0]))


def test_empty_span(orc):
    w = inputs.orbits_forward(n=2, seed=16)
    o = orc.solve(w["rhs"], "tsit5", w["y0"], w["theta"], 3.0, 3.0, 1e-8, 1e-10, [3.0])
    np.testing.assert_array_equal(o["y_final"], w["y0"])
    np.testing.assert_array_equal(o["y_out"][:, 0, :], w["y0"])
    assert np.all(o["n_accepted"] == 0)


def test_tolerance_proportionality(orc):
    """Global error falls as the tolerance is tightened (factor ~ tol ratio)."""
    w = inputs.orbits_forward(n=16, seed=17)
    ref = orc.solve(w["rhs"], "verner7", w["y0"], w["theta"], 0.0, 50.0, 1e-13, 1e-13)
    errs = []
    for tol in (1e-6, 1e-8, 1e-10):
        o = orc.solve(w["rhs"], "dopri5", w["y0"], w["theta"], 0.0, 50.0, tol, tol)
        errs.append(np.median(np.abs(o["y_final"] - ref["y_final"]).max(axis=0)))
    assert errs[0] > 10 * errs[1] > 100 * errs[2]
