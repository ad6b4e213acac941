"""Pins for the oracle's dark-energy profile (oracle/de_profile.py):
shooting for the flat amplitude (eq:de-flat), the implicit-function-theorem
derivative along flat models (eq:de-ift) and the Gauss-Newton fit (eq:de-gn).

lambda = 0 is a cosmological constant: the field never moves, the flat
amplitude is 1 - Om - Or with da0/dOm = -1, and distances are quadratures of
1/E with E^2 = Om (1+z)^3 + Or (1+z)^4 + 1 - Om - Or.
"""
import numpy as np
import pytest
from scipy.integrate import quad

from paper_2609_28458_amd import inputs

TIGHT = dict(tableau="dopri5", t0=-np.log(51.0), rtol=1e-11, atol=1e-13)


@pytest.fixture(scope="module")
def de(orc):
    from oracle import de_profile
    return de_profile


def test_shooting_makes_the_model_flat(de):
    rng = np.random.default_rng(3)
    lam, om = rng.uniform(0.0, 1.5, 12), rng.uniform(0.28, 0.34, 12)
    w = inputs.de_profile_mocks(n_mocks=1, n_lambda=1)
    s = dict(tableau="dopri5", t0=w["t0"], rtol=w["rtol"], atol=w["atol"])
    a0 = de.flat_amplitude(1.0 - om - w["omega_r"], lam, om, w["omega_r"], s, 4)
    _, _, _, _, e2, st = de.model(a0, lam, om, np.ones(12), w["omega_r"], w["N_nodes"], s)
    assert st == 0
    np.testing.assert_allclose(e2, 1.0, rtol=0, atol=1e-12)
    # a thawing field has used some of its energy: the flat amplitude is larger
    assert np.all(a0[lam > 0.1] > 1.0 - om[lam > 0.1] - w["omega_r"])


def test_cosmological_constant_closed_form(de):
    om = np.array([0.28, 0.31, 0.34])
    orad = 9.0e-5
    lam = np.zeros(3)
    z = np.array([2.33, 1.0, 0.3])  # nodes in increasing N = -ln(1+z)
    N = -np.log1p(z)
    a0 = de.flat_amplitude(1.0 - om - orad, lam, om, orad, TIGHT, 2)
    np.testing.assert_allclose(a0, 1.0 - om - orad, rtol=0, atol=1e-15)  # Om + Or + a0 = 1 to an ulp
    D, dDo, dDh, da0, _, _ = de.model(a0, lam, om, np.full(3, 2.0), orad, N, TIGHT)
    np.testing.assert_allclose(da0, -1.0, rtol=0, atol=1e-12)

    def E(zz, m):
        return np.sqrt(m * (1 + zz) ** 3 + orad * (1 + zz) ** 4 + 1.0 - m - orad)

    for i, m in enumerate(om):
        for k, zz in enumerate(z):
            dm = quad(lambda x: 1.0 / E(x, m), 0.0, zz, epsabs=1e-14, epsrel=1e-13)[0]
            ddm = quad(lambda x: -0.5 * ((1 + x) ** 3 - 1.0) / E(x, m) ** 3, 0.0, zz,
                       epsabs=1e-14, epsrel=1e-13)[0]
            assert abs(D[0, k, i] - dm / 2.0) < 1e-9
            assert abs(D[1, k, i] - 1.0 / (2.0 * E(zz, m))) < 1e-12
            assert abs(dDo[0, k, i] - ddm / 2.0) < 1e-8
            ddh = -0.5 * ((1 + zz) ** 3 - 1.0) / E(zz, m) ** 3 / 2.0
            assert abs(dDo[1, k, i] - ddh) < 1e-9
            assert abs(dDh[0, k, i] + D[0, k, i] / 2.0) < 1e-15


def test_flat_derivative_matches_reshooting(de):
    """da0/dOm and dD/dOm along flat models against central differences of
    re-shot models (tight tolerances so the adaptive steps barely move)."""
    lam = np.array([0.5, 1.2])
    om = np.array([0.30, 0.33])
    orad = 9.0e-5
    N = inputs.quintessence(n=1)["t_out"]
    a0 = de.flat_amplitude(1.0 - om - orad, lam, om, orad, TIGHT, 5)
    D, dDo, _, da0, _, _ = de.model(a0, lam, om, np.ones(2), orad, N, TIGHT)
    eps = 1e-5
    ap = de.flat_amplitude(a0, lam, om + eps, orad, TIGHT, 5)
    am = de.flat_amplitude(a0, lam, om - eps, orad, TIGHT, 5)
    np.testing.assert_allclose(da0, (ap - am) / (2 * eps), rtol=1e-5)
    Dp = de.model(ap, lam, om + eps, np.ones(2), orad, N, TIGHT)[0]
    Dm = de.model(am, lam, om - eps, np.ones(2), orad, N, TIGHT)[0]
    np.testing.assert_allclose(dDo, (Dp - Dm) / (2 * eps), rtol=2e-5, atol=1e-9)


def test_gauss_newton_recovers_noise_free_fiducial(de):
    w = inputs.de_profile_mocks(n_mocks=1, n_lambda=1)
    s = dict(tableau=w["tableau"], t0=w["t0"], rtol=w["rtol"], atol=w["atol"])
    f = w["fid"]
    orad = w["omega_r"]
    lam, om, h = np.array([f["lam"]]), np.array([f["om"]]), np.array([f["h"]])
    a0 = de.flat_amplitude(1.0 - om - orad, lam, om, orad, s, 4)
    D = de.model(a0, lam, om, h, orad, w["N_nodes"], s)[0]
    sigma = w["rel_noise"] * D[:, :, 0]
    st = w["start"]
    out = de.profile(lam, np.array([st["om"]]), np.array([st["h"]]),
                     np.array([1.0 - st["om"] - orad]), orad, w["N_nodes"], D, sigma, s,
                     iters=w["iters"], newton=w["newton"], mu=w["mu"], trust=w["trust"])
    assert abs(out["om"][0] - f["om"]) < 1e-7 and abs(out["h"][0] - f["h"]) < 1e-7
    assert out["chi2"][0] < 1e-10


def test_spline_reproduces_cubics_in_ln1pz(de):
    """A not-a-knot cubic spline is exact on cubic polynomials of its
    variable; a spline in z or with the nodes taken out of order is not."""
    N_nodes = inputs.quintessence(n=1, dense=True)["t_out"]
    N_data = inputs.quintessence(n=1)["t_out"]
    x_n, x_d = -N_nodes, -N_data

    def cubic(x):
        return np.stack([0.3 - 1.1 * x + 0.7 * x ** 2 - 0.45 * x ** 3,
                         2.0 + 0.2 * x - 0.9 * x ** 3])[:, :, None] * np.array([1.0, -2.0])

    got = de.at_data(cubic(x_n), N_nodes, N_data)
    np.testing.assert_allclose(got, cubic(x_d), rtol=0, atol=1e-13)
    assert de.at_data(cubic(x_n), N_nodes, None) is not None


def test_spline_profile_with_data_at_nodes_equals_direct(de):
    """With the data redshifts among the spline nodes the spline returns the
    node values, so the fit equals the fit with the nodes at the data (the
    solver's steps do not depend on the output times)."""
    w = inputs.de_profile_mocks(n_mocks=1, n_lambda=1)
    s = dict(tableau=w["tableau"], t0=w["t0"], rtol=w["rtol"], atol=w["atol"])
    orad = w["omega_r"]
    N_data = w["N_nodes"]
    N_nodes = np.unique(np.concatenate([N_data, w["N_spline"]]))
    lam = np.array([0.4, 1.3])
    om = np.array([0.30, 0.32])
    a0 = de.flat_amplitude(1.0 - om - orad, lam, om, orad, s, 4)
    D = de.model(a0, lam, om, np.ones(2), orad, N_data, s)[0] * 1.01
    sigma = 0.01 * D[:, :, 0]
    kw = dict(iters=4, newton=2, mu=w["mu"], trust=w["trust"])
    start = (np.full(2, 0.29), np.full(2, 0.98), 1.0 - np.full(2, 0.29) - orad)
    a = de.profile(lam, *start[:2], start[2], orad, N_data, D, sigma, s, **kw)
    b = de.profile(lam, *start[:2], start[2], orad, N_nodes, D, sigma, s, N_data=N_data, **kw)
    for k in ("om", "h", "a0", "chi2", "decrement"):
        np.testing.assert_allclose(b[k], a[k], rtol=1e-12, atol=1e-14)


def test_spline_distances_of_lcdm(de):
    """64-node spline of the distances at lambda = 0 against the quadratures
    at the 7 data redshifts: the spline error of smooth distances."""
    orad = 9.0e-5
    om = np.array([0.28, 0.34])
    lam = np.zeros(2)
    N_nodes = inputs.quintessence(n=1, dense=True)["t_out"]
    z_data = inputs.quintessence(n=1)["z_nodes"]
    a0 = 1.0 - om - orad
    D = de.at_data(de.model(a0, lam, om, np.ones(2), orad, N_nodes, TIGHT)[0], N_nodes,
                   -np.log1p(z_data))

    def E(zz, m):
        return np.sqrt(m * (1 + zz) ** 3 + orad * (1 + zz) ** 4 + 1.0 - m - orad)

    for i, m in enumerate(om):
        for k, zz in enumerate(z_data):
            dm = quad(lambda x: 1.0 / E(x, m), 0.0, zz, epsabs=1e-14, epsrel=1e-13)[0]
            assert abs(D[0, k, i] - dm) < 2e-7
            assert abs(D[1, k, i] - 1.0 / E(zz, m)) < 2e-7
