"""Pins of the oracle's forward sensitivities (eq:sens, eq:stage-sens).

On a fixed sequence of steps the integrated S is exactly the derivative of
the numerical solution (Appendix "Derivatives"), so it must equal central
finite differences of the same discrete map with the step sequence frozen.
The dual-number Jacobian of each right-hand side must equal finite
differences of its values, and for the harmonic oscillator dx/domega has a
closed form.
"""
import numpy as np
import pytest

from paper_2609_28458_amd import inputs

CASES = {
    "loghalo": (lambda: inputs.orbits_forward(n=6, seed=31), 0.0, 20.0, "dopri5", 1e-8, 1e-10),
    "spinprec": (lambda: inputs.spin_precession(n=4, seed=32), 100 ** -0.5, 30 ** -0.5,
                 "verner7", 1e-9, 1e-9),
    "quint": (lambda: inputs.quintessence(n=6, seed=33), -np.log(51.0), 0.0, "tsit5", 1e-8, 1e-11),
}


def _per_traj_theta(w, n):
    th = np.asarray(w["theta"], float)
    return th if th.ndim == 2 else np.repeat(th[:, None], n, axis=1)


@pytest.mark.parametrize("name", list(CASES))
def test_rhs_jacobian_matches_fd(orc, name):
    make, t0, t1, *_ = CASES[name]
    w = make()
    d, p = w["y0"].shape[0], _per_traj_theta(w, w["y0"].shape[1]).shape[0]
    rng = np.random.default_rng(0)
    y = w["y0"][:, 0] + 0.05 * rng.normal(size=d)
    th = _per_traj_theta(w, w["y0"].shape[1])[:, 0]
    t = 0.5 * (t0 + t1)
    cols = list(range(d + p))
    f, J = orc.rhs(name, t, y, th, cols)
    for c in cols:
        z = np.concatenate([y, th])
        eps = 1e-6 * max(1.0, abs(z[c]))
        zp, zm = z.copy(), z.copy()
        zp[c] += eps
        zm[c] -= eps
        fd = (orc.rhs(name, t, zp[:d], zp[d:]) - orc.rhs(name, t, zm[:d], zm[d:])) / (2 * eps)
        np.testing.assert_allclose(J[:, c], fd, rtol=1e-6, atol=1e-8 * np.max(np.abs(f)))


@pytest.mark.parametrize("name", list(CASES))
def test_sensitivities_equal_frozen_step_fd(orc, name):
    make, t0, t1, tab, rtol, atol = CASES[name]
    w = make()
    n = w["y0"].shape[1]
    d = w["y0"].shape[0]
    th = _per_traj_theta(w, n)
    p = th.shape[0]
    cols = list(range(d + p))
    nodes = np.linspace(t0, t1, 6)[1:-1]
    rec = orc.solve(name, tab, w["y0"], th, t0, t1, rtol, atol, nodes, h_cap=20000)
    fs = orc.solve(name, tab, w["y0"], th, t0, t1, rtol, atol, nodes, sens_cols=cols)
    # the sensitivity solve takes exactly the steps of the plain solve
    np.testing.assert_array_equal(fs["n_accepted"], rec["n_accepted"])
    np.testing.assert_array_equal(fs["y_final"], rec["y_final"])
    hs, nr = rec["h_rec"], rec["n_accepted"]
    def central(c, eps):
        outs = []
        for sgn in (+1, -1):
            y0 = w["y0"].copy()
            tt = th.copy()
            if c < d:
                y0[c] += sgn * eps
            else:
                tt[c - d] += sgn * eps
            outs.append(orc.solve(name, tab, y0, tt, t0, t1, rtol, atol, nodes,
                                  h_replay=hs, n_replay=nr))
        return ((outs[0]["y_final"] - outs[1]["y_final"]) / (2 * eps),
                (outs[0]["y_out"] - outs[1]["y_out"]) / (2 * eps))

    for c in cols:
        base = w["y0"][c] if c < d else th[c - d]
        eps = 2e-6 * np.maximum(1.0, np.abs(base))
        # Richardson extrapolation removes the O(eps^2) truncation error.
        f1, n1 = central(c, eps)
        f2, n2 = central(c, eps / 2)
        fdf, fdn = (4 * f2 - f1) / 3, (4 * n2 - n1) / 3
        scale = max(1.0, np.max(np.abs(fs["S_final"][:, c])))
        np.testing.assert_allclose(fs["S_final"][:, c], fdf, rtol=0, atol=1e-6 * scale)
        np.testing.assert_allclose(fs["S_out"][:, c], fdn, rtol=0, atol=1e-6 * scale)


def test_harmonic_closed_form_sensitivity(orc):
    x0, v0, w0, T = 0.7, -0.2, 1.3, 7.0
    nodes = np.array([1.0, 3.3, 6.1])
    o = orc.solve("harmonic", "verner7", np.array([[x0], [v0]]), np.array([w0]), 0.0, T, 1e-13,
                  1e-13, nodes, sens_cols=[0, 1, 2])
    t = nodes
    dx_dw = -x0 * t * np.sin(w0 * t) + v0 * (t * np.cos(w0 * t) / w0 - np.sin(w0 * t) / w0 ** 2)
    np.testing.assert_allclose(o["S_out"][0, 2, :, 0], dx_dw, atol=1e-10)
    np.testing.assert_allclose(o["S_out"][0, 0, :, 0], np.cos(w0 * t), atol=1e-11)
    np.testing.assert_allclose(o["S_out"][0, 1, :, 0], np.sin(w0 * t) / w0, atol=1e-11)
