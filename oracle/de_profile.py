"""Oracle for the dark-energy profile likelihood -- test infrastructure only.

Plain numpy on top of the oracle's ensemble solve with forward sensitivities
(``oracle.solve(..., sens_cols=...)``), one vectorised step at a time, in the
order of the paper's Section "A profile likelihood" and its appendix
"Data model and minimiser":

* the amplitude a0 of each model is fixed by flatness, g(a0) = E(0)^2 - 1 = 0
  (eq:de-flat), with Newton steps whose slope dg/da0 comes from the
  sensitivity S_a0 at N = 0 (the shooting method);
* the derivative along flat models follows the implicit-function theorem,
  da0/dOm = -(dg/dOm)/(dg/da0), dy/dOm = S_Om + (da0/dOm) S_a0 (eq:de-ift);
* distances D_M = (I(0) - I(N_z))/h and D_H = 1/(h E(N_z)) in units of the
  reference Hubble distance, h = H0 / H0_ref entering only as a scale;
* optionally (appendix "Data model and minimiser") the model distances at
  the data redshifts are read off a cubic spline in ln(1+z) through the node
  values; the spline is scipy's not-a-knot CubicSpline, a linear map, so the
  derivatives go through the same spline;
* whitened residuals r = (D_model - D_data)/sigma and the damped Gauss-Newton
  update psi <- psi - (J^T J + mu diag J^T J)^{-1} J^T r over psi = (Om, h)
  (eq:de-gn), the step scaled back into a box trust region; before each
  update's Newton steps the amplitude is moved with da0/dOm.

State y = (phi, u, I); theta = (a0, lambda, Om, Or).
"""
from __future__ import annotations

import numpy as np
from scipy.interpolate import CubicSpline

import oracle

A0, LAM, OM, OR = 0, 1, 2, 3          # theta rows
COL_A0, COL_OM = 3 + A0, 3 + OM        # sensitivity columns (d = 3)


def _theta(a0, lam, om, orad):
    return np.stack([a0, lam, om, np.broadcast_to(orad, np.shape(a0))]).astype(np.float64)


def _e2_parts(N, y, a0, lam, om, orad):
    """E^2 = Nm / Dn at e-fold N with Nm = Om e^{-3N} + Or e^{-4N} + a0
    e^{-lam phi}, Dn = 1 - u^2/6 (the Friedmann equation of eq:de-model)."""
    phi, u = y[0], y[1]
    ex = np.exp(-lam * phi)
    Nm = om * np.exp(-3.0 * N) + orad * np.exp(-4.0 * N) + a0 * ex
    Dn = 1.0 - u * u / 6.0
    return Nm, Dn, ex


def _de2(N, y, dy, a0, lam, om, orad, da0, dom):
    """Total derivative of E^2 at N along a direction in which the state moves
    by dy (phi, u components), a0 by da0 and Om by dom."""
    Nm, Dn, ex = _e2_parts(N, y, a0, lam, om, orad)
    u = y[1]
    dNm = np.exp(-3.0 * N) * dom + ex * da0 - lam * a0 * ex * dy[0]
    dDn = -u * dy[1] / 3.0
    return dNm / Dn - Nm * dDn / (Dn * Dn)


def _solve(theta, K_nodes, settings, cols):
    return oracle.solve("quint", settings["tableau"], np.zeros((3, theta.shape[1])), theta,
                        settings["t0"], 0.0, settings["rtol"], settings["atol"], K_nodes,
                        sens_cols=cols)


def flat_amplitude(a0, lam, om, orad, settings, newton):
    """`newton` Newton steps on g(a0) = E(0)^2 - 1 from a0 (eq:de-flat)."""
    a0 = np.array(a0, dtype=np.float64)
    for _ in range(newton):
        o = _solve(_theta(a0, lam, om, orad), None, settings, [COL_A0])
        y, S = o["y_final"], o["S_final"][:, 0]
        Nm, Dn, _ = _e2_parts(0.0, y, a0, lam, om, orad)
        g = Nm / Dn - 1.0
        dg = _de2(0.0, y, S, a0, lam, om, orad, 1.0, 0.0)
        a0 = a0 - g / dg
    return a0


def model(a0, lam, om, h, orad, N_nodes, settings):
    """Distances at the nodes and their derivatives with respect to psi =
    (Om, h) along flat models.  Returns D [2][K][n] (D_M, D_H), dD/dOm,
    dD/dh, da0/dOm, E(0)^2 and the worst solver status."""
    o = _solve(_theta(a0, lam, om, orad), N_nodes, settings, [COL_A0, COL_OM])
    yf, Sf = o["y_final"], o["S_final"]
    # implicit-function theorem at N = 0 (eq:de-ift)
    dg_a0 = _de2(0.0, yf, Sf[:, 0], a0, lam, om, orad, 1.0, 0.0)
    dg_om = _de2(0.0, yf, Sf[:, 1], a0, lam, om, orad, 0.0, 1.0)
    da0 = -dg_om / dg_a0
    dyf = Sf[:, 1] + da0 * Sf[:, 0]                     # dy(0)/dOm along flat models
    yo, So = o["y_out"], o["S_out"]                     # [3][K][n], [3][2][K][n]
    dyo = So[:, 1] + da0[None, :] * So[:, 0]            # [3][K][n]
    N = np.asarray(N_nodes, dtype=np.float64)[:, None]
    DM = (yf[2][None, :] - yo[2]) / h
    dDM = (dyf[2][None, :] - dyo[2]) / h
    Nm, Dn, _ = _e2_parts(N, yo, a0, lam, om, orad)
    E = np.sqrt(Nm / Dn)
    DH = 1.0 / (h * E)
    dE2 = _de2(N, yo, dyo, a0, lam, om, orad, da0, 1.0)
    dDH = -0.5 * dE2 / (h * E ** 3)
    D = np.stack([DM, DH])
    dD_om = np.stack([dDM, dDH])
    Nm0, Dn0, _ = _e2_parts(0.0, yf, a0, lam, om, orad)
    return D, dD_om, -D / h, da0, Nm0 / Dn0, int(o["status"].max())


def at_data(Dnode, N_nodes, N_data):
    """Node values [2][K][n] -> values at the data e-folds [2][Kd][n] by a
    not-a-knot cubic spline in x = ln(1+z) = -N (None: the data sit at the
    nodes)."""
    if N_data is None:
        return Dnode
    x = -np.asarray(N_nodes, dtype=np.float64)
    order = np.argsort(x)
    spl = CubicSpline(x[order], Dnode[:, order, :], axis=1)
    return spl(-np.asarray(N_data, dtype=np.float64))


def profile(lam, om, h, a0, orad, N_nodes, data, sigma, settings, iters=20, newton=3,
            mu=1e-3, trust=(0.05, 0.05), N_data=None):
    """Damped Gauss-Newton fits of psi = (Om, h) at fixed lam (one per column
    of the inputs), a0 solved by shooting.  data [2][Kd][n], sigma [2][Kd]
    at the nodes (Kd = K) or, with N_data [Kd], at those e-folds through the
    spline of `at_data`.  Returns a dict: om, h, a0 (flat at the returned
    parameters), chi2 there, chi2_prev (before the last update), decrement
    (last g^T step), dist (the model distances at the data points at the
    returned parameters)."""
    om = np.array(om, dtype=np.float64)
    h = np.array(h, dtype=np.float64)
    a0 = np.array(a0, dtype=np.float64)
    sig = np.asarray(sigma, dtype=np.float64)[:, :, None]
    chi2_prev = np.full(om.shape, np.nan)
    dec = np.full(om.shape, np.nan)
    for _ in range(iters):
        a0 = flat_amplitude(a0, lam, om, orad, settings, newton)
        D, dDo, _, da0, _, _ = model(a0, lam, om, h, orad, N_nodes, settings)
        D, dDo = at_data(D, N_nodes, N_data), at_data(dDo, N_nodes, N_data)
        dDh = -D / h
        r = ((D - data) / sig).reshape(-1, om.size)
        J = np.stack([(dDo / sig).reshape(-1, om.size), (dDh / sig).reshape(-1, om.size)])
        A11 = np.sum(J[0] * J[0], axis=0)
        A12 = np.sum(J[0] * J[1], axis=0)
        A22 = np.sum(J[1] * J[1], axis=0)
        g1 = np.sum(J[0] * r, axis=0)
        g2 = np.sum(J[1] * r, axis=0)
        B11, B22 = A11 * (1.0 + mu), A22 * (1.0 + mu)
        det = B11 * B22 - A12 * A12
        s1 = (B22 * g1 - A12 * g2) / det
        s2 = (B11 * g2 - A12 * g1) / det
        # scale the step back into the trust box |dOm| <= trust[0], |dh| <= trust[1]
        f = np.minimum(1.0, np.minimum(trust[0] / np.maximum(np.abs(s1), 1e-300),
                                       trust[1] / np.maximum(np.abs(s2), 1e-300)))
        s1, s2 = f * s1, f * s2
        chi2_prev = np.sum(r * r, axis=0)
        dec = g1 * s1 + g2 * s2
        om = om - s1
        h = h - s2
        a0 = a0 - da0 * s1          # move the amplitude to the new Om
    a0 = flat_amplitude(a0, lam, om, orad, settings, newton)
    D, _, _, _, _, st = model(a0, lam, om, h, orad, N_nodes, settings)
    D = at_data(D, N_nodes, N_data)
    chi2 = np.sum((((D - data) / sig) ** 2).reshape(-1, om.size), axis=0)
    return dict(om=om, h=h, a0=a0, chi2=chi2, chi2_prev=chi2_prev, decrement=dec, dist=D,
                status=st)
