"""Pins of the oracle's Butcher tableaux against what the mathematics fixes.

The paper names the methods and their orders (Appendix "Runge--Kutta steps
and error control": Tsit5 and Dopri5 of order 5, Verner 7 of order 7, the
embedded estimate one order lower) and the interpolant property b_j(1) = b_j
(Appendix "Dense output").  The coefficients themselves are transcribed from
the primary publications; these tests make a mistyped digit fail.
"""
import mpmath as mp
import numpy as np
import pytest

from rk_trees import gamma, order, phi, residual_at, residuals, trees

mp.mp.dps = 40
NAMES = ["dopri5", "tsit5", "verner7"]
ORDER = {"dopri5": 5, "tsit5": 5, "verner7": 7}
STAGES = {"dopri5": 7, "tsit5": 7, "verner7": 10}


def mpm(x):
    return [[mp.mpf(float(v)) for v in row] for row in x]


def test_tree_counts():
    assert [len(trees(n)) for n in range(1, 9)] == [1, 1, 2, 4, 9, 20, 48, 115]
    # gamma of the bushy tree of order n is n, of the tall tree n!
    assert gamma(((), (), ())) == 4
    assert gamma(((((),),),)) == 24


@pytest.mark.parametrize("name", NAMES)
def test_shape_and_row_sums(orc, name):
    T = orc.tableau(name)
    assert T["s"] == STAGES[name] and T["order"] == ORDER[name]
    a, c = T["a"], T["c"]
    assert np.all(np.triu(a) == 0.0), "explicit method: strictly lower-triangular A"
    np.testing.assert_allclose(a.sum(axis=1), c, atol=2e-15)
    assert abs(T["b"].sum() - 1.0) < 1e-15
    assert abs(T["bdiff"].sum()) < 1e-15


@pytest.mark.parametrize("name", NAMES)
def test_order_conditions(orc, name):
    """b has order nu, bhat = b - bdiff order nu - 1, and neither one more."""
    T = orc.tableau(name)
    nu = T["order"]
    A = mpm(T["a"])
    b = [mp.mpf(float(v)) for v in T["b"]]
    bh = [mp.mpf(float(v)) - mp.mpf(float(e)) for v, e in zip(T["b"], T["bdiff"])]
    assert residuals(A, b, nu) < 1e-13
    assert residuals(A, bh, nu - 1) < 1e-13
    assert residual_at(A, b, nu + 1) > 1e-6
    assert residual_at(A, bh, nu) > 1e-6


def test_dopri5_matches_scipy(orc):
    """Dopri5 coefficients and continuous extension equal scipy's RK45 arrays."""
    from scipy.integrate._ivp.rk import RK45

    T = orc.tableau("dopri5")
    np.testing.assert_allclose(T["c"][:6], RK45.C, rtol=0, atol=1e-16)
    np.testing.assert_allclose(T["a"][:6, :5], RK45.A, rtol=0, atol=2e-15)
    np.testing.assert_allclose(T["b"][:6], RK45.B, rtol=0, atol=1e-16)
    # scipy stores E = bhat - b (opposite sign convention), FSAL stage last.
    np.testing.assert_allclose(T["bdiff"], -RK45.E, rtol=0, atol=1e-16)
    np.testing.assert_allclose(T["P"], RK45.P, rtol=0, atol=2e-15)


@pytest.mark.parametrize("name", ["dopri5", "tsit5"])
def test_dense_interpolant(orc, name):
    """b_j(1) = b_j and the interpolant has order 4 for every sigma."""
    T = orc.tableau(name)
    P = T["P"]
    w1 = P.sum(axis=1)
    np.testing.assert_allclose(w1, T["b"], atol=2e-14)
    A = mpm(T["a"])
    for sig in ["0.1", "0.37", "0.5", "0.83"]:
        s = mp.mpf(sig)
        bs = [mp.fsum(mp.mpf(float(P[j][k])) * s ** (k + 1) for k in range(P.shape[1]))
              for j in range(T["s"])]
        worst = mp.mpf(0)
        for n in range(1, 5):
            for t in trees(n):
                g = phi(t, A)
                worst = max(worst, abs(mp.fsum(bs[i] * g[i] for i in range(T["s"]))
                                       - s ** n / gamma(t)))
        assert worst < 1e-13, (sig, worst)


def test_fsal_structure(orc):
    for name in ["dopri5", "tsit5"]:
        T = orc.tableau(name)
        assert T["fsal"] and T["c"][-1] == 1.0
        np.testing.assert_array_equal(T["a"][-1, :], T["b"])
    assert not orc.tableau("verner7")["fsal"]
