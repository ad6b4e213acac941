"""Pins for the oracle's stiff path (oracle/stiff.cpp): Rodas4 in the textbook
form of a Rosenbrock method (Hairer & Wanner 1996, Sec. IV.7) on the stiff
kinetics networks kin3 and kin8.

- the standard-form coefficients the oracle derives from the published
  transformed ones satisfy the Rosenbrock order conditions of order 4 (and
  3 for the embedded solution), with the method's rounded nodes;
- the stability function vanishes at infinity and is bounded by 1 in the
  left half-plane (stiffly accurate, L-stable);
- fixed steps converge at order 4;
- a linear network equals the matrix exponential (scipy.linalg.expm);
- adaptive solutions agree with scipy's Radau at tight tolerances within the
  requested tolerance, and the linear invariants of both networks hold to
  rounding;
- the hand-written Jacobians equal central differences.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm

from paper_2609_28458_amd import inputs


@pytest.fixture(scope="module")
def rc(orc):
    return orc.rodas4()


def _conds(b, alpha, Gam, g):
    """Order conditions of a Rosenbrock method up to order 4 (beta = alpha +
    the strictly lower part of Gamma; alpha_i, beta_i row sums)."""
    beta = alpha + np.tril(Gam, -1)
    al, be = alpha.sum(1), beta.sum(1)
    return np.array([
        b.sum() - 1.0,
        b @ be - (0.5 - g),
        b @ al ** 2 - 1.0 / 3.0,
        b @ beta @ be - (1.0 / 6.0 - g + g * g),
        b @ al ** 3 - 0.25,
        b @ (al * (alpha @ be)) - (1.0 / 8.0 - g / 3.0),
        b @ beta @ al ** 2 - (1.0 / 12.0 - g / 3.0),
        b @ beta @ beta @ be - (1.0 / 24.0 - g / 2.0 + 1.5 * g * g - g ** 3),
    ])


def test_rodas4_order_conditions(rc):
    g = rc["gamma"]
    assert g == 0.25
    assert np.allclose(np.diag(rc["Gamma"]), g, rtol=0, atol=1e-15)
    assert np.all(np.triu(rc["alpha"]) == 0.0) and np.all(np.triu(rc["Gamma"], 1) == 0.0)
    main = _conds(rc["b"], rc["alpha"], rc["Gamma"], g)
    emb = _conds(rc["bhat"], rc["alpha"], rc["Gamma"], g)
    assert np.max(np.abs(main)) < 1e-13, main
    assert np.max(np.abs(emb[:4])) < 1e-13, emb
    assert np.max(np.abs(emb[4:])) > 1e-3  # the embedded solution is of order 3 only
    # the method's nodes and gamma_i (row sums), rounded as published
    np.testing.assert_allclose(rc["alpha"].sum(1), [0.0, 0.386, 0.21, 0.63, 1.0, 1.0],
                               atol=1e-14)
    np.testing.assert_allclose(rc["Gamma"].sum(1), [0.25, -0.1043, 0.1035, -0.0362, 0.0, 0.0],
                               atol=1e-14)


def _R(z, rc):
    B = rc["alpha"] + rc["Gamma"]
    one = np.ones(6)
    return 1.0 + z * rc["b"] @ np.linalg.solve(np.eye(6) - z * B, one)


def test_rodas4_is_l_stable(rc):
    assert abs(_R(-1e12, rc)) < 1e-9
    for y in np.linspace(-200.0, 200.0, 801):
        assert abs(_R(1j * y, rc)) <= 1.0 + 1e-12
    rng = np.random.default_rng(0)
    z = -np.exp(rng.uniform(-3, 8, 400)) + 1j * rng.normal(0, 50, 400)
    assert max(abs(_R(x, rc)) for x in z) <= 1.0 + 1e-12
    # order 4: R(z) - e^z = O(z^5), so halving z divides the difference by ~32
    for z in (0.2, -0.2, 0.2j):
        ratio = abs(_R(z, rc) - np.exp(z)) / abs(_R(z / 2, rc) - np.exp(z / 2))
        assert 25.0 < ratio < 40.0, ratio


def _one(orc, rhs, y0, th, t1, **kw):
    o = orc.solve(rhs, "rodas4", np.asarray(y0, float)[:, None], np.asarray(th, float)[:, None],
                  0.0, t1, kw.pop("rtol", 1e-6), kw.pop("atol", 1e-10), **kw)
    return o


def test_fixed_steps_converge_at_order_4(orc):
    """Mild rates (no stiffness) and constant steps: the global error falls
    as h^4."""
    th = np.array([1.0, 10.0, 2.0])
    y0 = np.array([0.6, 0.1, 0.3])
    t1 = 2.0
    f = lambda t, y: orc.stiff_rhs("kin3", y, th)[0]
    ref = solve_ivp(f, (0, t1), y0, method="DOP853", rtol=1e-13, atol=1e-15).y[:, -1]
    errs = []
    for N in (10, 20, 40, 80):
        o = _one(orc, "kin3", y0, th, t1, h0=t1 / N, alpha_min=1.0, alpha_max=1.0, safety=1.0,
                 rtol=1e10, atol=1e10)
        assert o["n_accepted"][0] in (N, N + 1)
        errs.append(np.max(np.abs(o["y_final"][:, 0] - ref)))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(slopes > 3.7) and np.all(slopes < 4.6), (errs, slopes)


def test_linear_network_equals_matrix_exponential(orc):
    """kin8 without the bilinear step (k6 = 0) is linear with a constant
    source: y(t) from the exponential of the augmented matrix."""
    th = inputs.KIN8_NOMINAL.copy()
    th[5] = 0.0
    y0 = np.array([1.0, 0.0, 0.2, 0.0, 1e-3, 0.1, 0.0, 0.0])
    f0, L = orc.stiff_rhs("kin8", np.zeros(8), th)
    Aug = np.zeros((9, 9))
    Aug[:8, :8] = L
    Aug[:8, 8] = f0  # f(y) = L y + f(0)
    t_out = np.array([0.0, 1e-3, 0.5, 7.0, 80.0, 300.0])
    o = _one(orc, "kin8", y0, th, 300.0, rtol=1e-10, atol=1e-14, t_out=t_out)
    assert o["status"][0] == 0
    for k, t in enumerate(t_out):
        exact = (expm(Aug * t) @ np.append(y0, 1.0))[:8]
        np.testing.assert_allclose(o["y_out"][:, k, 0], exact, rtol=1e-7, atol=1e-12)
    np.testing.assert_array_equal(o["y_out"][:, 0, 0], y0)       # node at t0 takes y0
    np.testing.assert_array_equal(o["y_out"][:, -1, 0], o["y_final"][:, 0])  # node at t1


@pytest.mark.parametrize("gen", [inputs.kinetics3, inputs.kinetics8], ids=["kin3", "kin8"])
def test_adaptive_solution_within_tolerance_of_radau(orc, gen):
    w = gen(n=12, seed=11)
    o = orc.solve(w["rhs"], "rodas4", w["y0"], w["theta"], w["t0"], w["t1"], w["rtol"],
                  w["atol"], w["t_out"])
    assert np.all(o["status"] == 0)
    assert o["n_accepted"].max() < 1000  # stiff: far below any explicit stability limit
    worst = 0.0
    for i in range(w["y0"].shape[1]):
        th = w["theta"][:, i]
        f = lambda t, y: orc.stiff_rhs(w["rhs"], y, th)[0]
        jac = lambda t, y: orc.stiff_rhs(w["rhs"], y, th)[1]
        r = solve_ivp(f, (0.0, w["t1"][i]), w["y0"][:, i], method="Radau", jac=jac, rtol=1e-12,
                      atol=1e-16, t_eval=w["t_out"][:, i])
        sc = w["atol"] + w["rtol"] * np.abs(r.y)
        worst = max(worst, np.max(np.abs(o["y_out"][:, :, i] - r.y) / sc))
    assert worst < 5.0, worst


@pytest.mark.parametrize("gen", [inputs.kinetics3, inputs.kinetics8], ids=["kin3", "kin8"])
def test_invariants_hold(orc, gen):
    w = gen(n=500, seed=12)
    o = orc.solve(w["rhs"], "rodas4", w["y0"], w["theta"], w["t0"], w["t1"], w["rtol"],
                  w["atol"], w["t_out"])
    keep = slice(None) if w["rhs"] == "kin3" else [0, 1, 2, 3, 5, 6, 7]
    inv0 = w["y0"][keep].sum(0)
    np.testing.assert_allclose(o["y_final"][keep].sum(0), inv0, rtol=0, atol=1e-13)
    np.testing.assert_allclose(o["y_out"][keep].sum(0), np.broadcast_to(inv0, o["y_out"].shape[1:]),
                               rtol=0, atol=1e-13)


@pytest.mark.parametrize("rhs,gen", [("kin3", inputs.kinetics3), ("kin8", inputs.kinetics8)])
def test_jacobian_matches_central_differences(orc, rhs, gen):
    w = gen(n=4, seed=13)
    rng = np.random.default_rng(1)
    for i in range(4):
        th = w["theta"][:, i]
        y = rng.uniform(0.0, 1.0, w["y0"].shape[0])
        _, J = orc.stiff_rhs(rhs, y, th)
        for j in range(len(y)):
            e = np.zeros_like(y)
            e[j] = 1e-6
            fd = (orc.stiff_rhs(rhs, y + e, th)[0] - orc.stiff_rhs(rhs, y - e, th)[0]) / 2e-6
            np.testing.assert_allclose(J[:, j], fd, rtol=1e-6, atol=1e-7 * np.abs(th).max())


def test_max_steps_reports_and_fills_nan(orc):
    w = inputs.kinetics3(n=3, seed=14)
    o = orc.solve(w["rhs"], "rodas4", w["y0"], w["theta"], w["t0"], w["t1"], w["rtol"],
                  w["atol"], w["t_out"], max_steps=5)
    assert np.all(o["status"] == 1)
    assert np.all(o["n_accepted"] + o["n_rejected"] == 5)
    assert np.isnan(o["y_out"][:, -1]).all()


# ---------------------------------------------------------------------------
# The two classic stiff chemistry problems (Robertson 1966; Schaefer 1975)
# in their textbook form (Hairer & Wanner 1996, Sec. IV.1 and IV.10),
# transcribed here a second time in numpy, independently of the oracle.

def rober_np(k):
    k1, k2, k3 = k

    def f(t, y):
        return np.array([-k1 * y[0] + k3 * y[1] * y[2],
                         k1 * y[0] - k3 * y[1] * y[2] - k2 * y[1] ** 2,
                         k2 * y[1] ** 2])
    return f


def hires_np(k):
    a, b, c, s, d, e, kf, g = k

    def f(t, y):
        r = kf * y[5] * y[7]
        return np.array([-a * y[0] + b * y[1] + c * y[2] + s,
                         a * y[0] - (b + c) * y[1],
                         -(a + c) * y[2] + b * y[3] + d * y[4],
                         c * y[1] + a * y[2] - e * y[3],
                         -(a + d) * y[4] + b * y[5] + b * y[6],
                         -r + g * y[3] + a * y[4] - b * y[5] + g * y[6],
                         r - (e + g) * y[6],
                         -r + (e + g) * y[6]])
    return f


TEXTBOOK = [("rober", inputs.robertson, rober_np), ("hires", inputs.hires, hires_np)]


def test_textbook_constants():
    """With the nominal constants the parameterised HIRES is the textbook
    problem: its other four rate constants are the sums 8.75, 10.03, 1.745,
    1.81 of the independent ones."""
    a, b, c, s, d, e, kf, g = inputs.HIRES_NOMINAL
    np.testing.assert_allclose([c + b, c + a, a + d, e + g], [8.75, 10.03, 1.745, 1.81],
                               rtol=1e-15)
    assert s == 0.0007 and kf == 280.0
    np.testing.assert_array_equal(inputs.ROBER_NOMINAL, [0.04, 3.0e7, 1.0e4])


@pytest.mark.parametrize("name,gen,fnp", TEXTBOOK, ids=["rober", "hires"])
def test_rhs_equals_the_textbook_form(orc, name, gen, fnp):
    w = gen(n=6, seed=21)
    rng = np.random.default_rng(4)
    for i in range(6):
        th = w["theta"][:, i]
        y = rng.uniform(0.0, 1.0, w["y0"].shape[0]) * (1e-3 if name == "hires" else 1.0)
        f, J = orc.stiff_rhs(name, y, th)
        np.testing.assert_allclose(f, fnp(th)(0.0, y), rtol=1e-14, atol=1e-18)
        for j in range(len(y)):
            ej = np.zeros_like(y)
            ej[j] = 1e-7 * max(abs(y[j]), 1e-3)
            fd = (orc.stiff_rhs(name, y + ej, th)[0] - orc.stiff_rhs(name, y - ej, th)[0]) / (
                2 * ej[j])
            np.testing.assert_allclose(J[:, j], fd, rtol=1e-6, atol=1e-8 * np.abs(th).max())


@pytest.mark.parametrize("name,gen,fnp", TEXTBOOK, ids=["rober", "hires"])
def test_textbook_problems_against_radau(orc, name, gen, fnp):
    """The oracle at a tight tolerance against scipy's Radau (called as a
    library, with the numpy transcription of the problem): agreement within
    the tighter of the two tolerances, at every output time."""
    w = gen(n=4, seed=22)
    rtol, atol = 1e-10, 1e-15
    o = orc.solve(name, "rodas4", w["y0"], w["theta"], 0.0, w["t1"], rtol, atol, w["t_out"])
    assert np.all(o["status"] == 0)
    worst = 0.0
    for i in range(4):
        th = w["theta"][:, i]
        t1 = float(np.broadcast_to(w["t1"], (4,))[i])
        t_out = w["t_out"][:, i] if np.ndim(w["t_out"]) == 2 else w["t_out"]
        r = solve_ivp(fnp(th), (0.0, t1), w["y0"][:, i], method="Radau", rtol=1e-12,
                      atol=1e-17, t_eval=t_out)
        assert r.success
        worst = max(worst, np.max(np.abs(o["y_out"][:, :, i] - r.y) / (atol + rtol * np.abs(r.y))))
    print(f"{name}: worst error vs Radau {worst:.2f} tolerance units")
    assert worst < 5.0, worst


@pytest.mark.parametrize("name,gen,fnp", TEXTBOOK, ids=["rober", "hires"])
def test_textbook_problems_linear_invariants(orc, name, gen, fnp):
    """Robertson keeps y1 + y2 + y3 = 1 and HIRES keeps y7 + y8 = 0.0057: a
    Rosenbrock method with the exact Jacobian preserves linear invariants, so
    they hold to rounding at the workload tolerance."""
    w = gen(n=300, seed=23)
    o = orc.solve(name, "rodas4", w["y0"], w["theta"], 0.0, w["t1"], w["rtol"], w["atol"],
                  w["t_out"])
    assert np.all(o["status"] == 0)
    rows = [0, 1, 2] if name == "rober" else [6, 7]
    inv0 = w["y0"][rows].sum(0)
    np.testing.assert_allclose(o["y_final"][rows].sum(0), inv0, rtol=0, atol=1e-14)
    np.testing.assert_allclose(o["y_out"][rows].sum(0),
                               np.broadcast_to(inv0, o["y_out"].shape[1:]), rtol=0, atol=1e-14)
    assert o["n_accepted"].max() < 1000  # stiff: far below any explicit stability limit
