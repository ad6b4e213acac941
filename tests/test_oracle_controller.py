"""Pin of the oracle's step-size controller in its PI form (eq:controller
generalised by reading c2), independent of the oracle's stage code.

On the linear system y' = A y (the harmonic oscillator, A = [[0, 1],
[-w^2, 0]]) one explicit Runge--Kutta step of length h is a matrix
polynomial: with the Butcher matrix a and weights w,

    h sum_j w_j k_j = sum_{m>=0} (w^T a^m 1) (hA)^(m+1) y,

so y+ = R(hA) y and the embedded error e = E(hA) y follow from the tableau
alone (a is strictly lower triangular, so the sum ends at m = s - 1).  The
test runs the controller of the reading on those exact step maps:

    factor = min(a_max, max(a_min, safety ||e||^(-beta1) ||e_prev||^beta2)),

||e_prev|| the norm of the last ACCEPTED step floored at 1e-4 (1 before
the first), factor a_max for ||e|| = 0, accept iff ||e|| <= 1, the last step
clipped to t1, and compares the accepted step sizes and the counts with the
oracle's.  Dopri5's coefficients come from scipy's RK45 (a source outside this
repository); Tsit5's and Verner 7's from the oracle's tables, which the
order-condition tests pin.  Each plausible slip in the PI branch (e_prev
updated on a rejection, the floor dropped, the sign of beta2 flipped, the
initial e_prev not 1) is run through the same simulation and must change the
accepted steps, so the comparison would catch it.
"""
import numpy as np
import pytest

OMEGA = 1.3
Y0 = np.array([1.0, 0.3])


def _weights(name, orc):
    if name == "dopri5":
        from scipy.integrate._ivp.rk import RK45

        s = 7
        a = np.zeros((s, s))
        a[:6, :5] = RK45.A
        a[6, :6] = RK45.B  # the FSAL row
        b = np.zeros(s)
        b[:6] = RK45.B
        bdiff = -RK45.E  # scipy stores bhat - b
        return a, b, bdiff, 5
    T = orc.tableau(name)
    return T["a"], T["b"], T["bdiff"], T["order"]


def _step_maps(a, w):
    """Coefficients g_m = w^T a^m 1 of the step polynomial sum g_m Z^(m+1)."""
    s = a.shape[0]
    v = np.ones(s)
    g = []
    for _ in range(s):
        g.append(float(w @ v))
        v = a @ v
    return g


def _apply(g, hA, y):
    out = np.zeros_like(y)
    Zp = hA.copy()
    for gm in g:
        out = out + gm * (Zp @ y)
        Zp = Zp @ hA
    return out


def simulate(name, orc, *, h0, t1, rtol, atol, safety=0.9, amin=0.2, amax=5.0, beta1=None,
             beta2=0.0, variant=None):
    """Accepted step sizes, counts and norms of the controller on y' = A y."""
    a, b, bdiff, order = _weights(name, orc)
    gb, ge = _step_maps(a, b), _step_maps(a, bdiff)
    A = np.array([[0.0, 1.0], [-OMEGA * OMEGA, 0.0]])
    b1 = 1.0 / order if beta1 is None else beta1
    t, y, h = 0.0, Y0.copy(), h0
    ep = 2.0 if variant == "start_not_one" else 1.0
    hs, norms, nrej = [], [], 0
    # a slip can stall the controller: give up after as many attempts as
    # any correct case needs ten times over
    while len(norms) < 20000 and h > 1e-14:
        last = t + h >= t1
        if last:
            h = t1 - t
        yn = y + _apply(gb, h * A, y)
        e = _apply(ge, h * A, y)
        sc = atol + rtol * np.maximum(np.abs(y), np.abs(yn))
        en = float(np.sqrt(np.mean((e / sc) ** 2)))
        norms.append(en)
        b2 = -beta2 if variant == "beta2_sign" else beta2
        if en == 0.0:
            factor = amax
        else:
            raw = safety * en ** (-b1) * ep ** b2
            factor = min(amax, max(amin, raw))
        if en <= 1.0:
            hs.append(h)
            t = t1 if last else t + h
            y = yn
            ep = en if variant == "no_floor" else max(en, 1e-4)
            if last:
                break
        else:
            nrej += 1
            if variant == "update_on_reject":
                ep = max(en, 1e-4)
        h = h * factor
    return np.array(hs), nrej, np.array(norms), y


def max_rel(a, b):
    """Largest relative difference of two step sequences (inf if their
    lengths differ)."""
    a, b = np.asarray(a), np.asarray(b)
    if a.shape != b.shape:
        return np.inf
    return float(np.max(np.abs(a - b) / np.abs(b)))


CASES = [
    # a first step far too long (rejections first), a PI controller
    dict(h0=4.0, t1=30.0, rtol=1e-7, atol=1e-9),
    # a first step far too short: norms below the 1e-4 floor, then growth
    dict(h0=1e-5, t1=30.0, rtol=1e-7, atol=1e-9),
]
PI = {"dopri5": (0.7 / 5, 0.4 / 5), "tsit5": (0.7 / 5, 0.4 / 5), "verner7": (0.7 / 7, 0.4 / 7)}


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("name", ["dopri5", "tsit5", "verner7"])
def test_pi_controller_step_sequence(orc, name, case):
    kw = CASES[case]
    b1, b2 = PI[name]
    hs, nrej, norms, yend = simulate(name, orc, beta1=b1, beta2=b2, **kw)
    # No attempt sits within rounding of the acceptance threshold, so the
    # oracle's stage-by-stage arithmetic must take the same decisions.
    assert np.min(np.abs(norms - 1.0)) > 1e-6
    o = orc.solve("harmonic", name, Y0.reshape(2, 1), np.array([OMEGA]), 0.0, kw["t1"],
                  kw["rtol"], kw["atol"], h0=kw["h0"], beta1=b1, beta2=b2, h_cap=4096)
    n = int(o["n_accepted"][0])
    assert o["status"][0] == 0
    assert n == len(hs) and int(o["n_rejected"][0]) == nrej
    # The error estimate is a difference of nearly equal terms, so the two
    # evaluation orders round it differently (relatively more the shorter
    # the step); through ||e||^(-beta1) that moves steps by up to ~1e-6
    # relative, and the differences wander over a few hundred steps.  Every
    # slip below changes some step by more than a per cent.
    assert max_rel(o["h_rec"][0, :n], hs) < 1e-4
    np.testing.assert_allclose(o["y_final"][:, 0], yend, rtol=0, atol=1e-7)


@pytest.mark.parametrize("name", ["dopri5", "tsit5", "verner7"])
def test_every_slip_changes_the_steps(orc, name):
    """Each plausible slip in the PI branch changes the accepted steps of at
    least one case by more than a per cent (or the counts), so the
    comparisons above would catch it."""
    b1, b2 = PI[name]
    ref = [simulate(name, orc, beta1=b1, beta2=b2, **kw) for kw in CASES]
    assert ref[0][1] >= 1, "case 0 has rejections"
    assert np.min(ref[1][2]) < 1e-4, "case 1 has norms below the floor"
    for variant in ("update_on_reject", "no_floor", "beta2_sign", "start_not_one"):
        caught = False
        for kw, (hs, nrej, _, _) in zip(CASES, ref):
            hv, nv, _, _ = simulate(name, orc, beta1=b1, beta2=b2, variant=variant, **kw)
            caught = caught or nv != nrej or max_rel(hv, hs) > 1e-2
        assert caught, f"{variant} leaves the accepted steps unchanged"


@pytest.mark.parametrize("name", ["dopri5", "verner7"])
def test_wide_clamp_and_safety(orc, name):
    """Non-default safety and clamp bounds (safety 0.5, alpha_min 0.05,
    alpha_max 200) with the I controller: the same matrix-polynomial pin, from
    a first step long enough to be cut by alpha_min."""
    kw = dict(h0=3.0, t1=20.0, rtol=1e-8, atol=1e-10)
    ctl = dict(safety=0.5, amin=0.05, amax=200.0)
    hs, nrej, norms, yend = simulate(name, orc, **ctl, **kw)
    assert nrej >= 1 and np.min(np.abs(norms - 1.0)) > 1e-6
    o = orc.solve("harmonic", name, Y0.reshape(2, 1), np.array([OMEGA]), 0.0, kw["t1"],
                  kw["rtol"], kw["atol"], h0=kw["h0"], safety=0.5, alpha_min=0.05,
                  alpha_max=200.0, h_cap=4096)
    n = int(o["n_accepted"][0])
    assert n == len(hs) and int(o["n_rejected"][0]) == nrej
    assert max_rel(o["h_rec"][0, :n], hs) < 1e-4
    # the default clamp gives other steps
    hd, nd, _, _ = simulate(name, orc, **kw)
    assert nd != nrej or max_rel(hd, hs) > 1e-2


def test_zero_error_grows_by_a_wide_alpha_max(orc):
    """f = 0 (omega = 0): every norm is exactly 0, so every accepted step
    grows by exactly alpha_max = 200 until the landing step."""
    o = orc.solve("harmonic", "verner7", np.zeros((2, 1)), np.array([0.0]), 0.0, 1e9, 1e-6,
                  1e-6, h0=1e-3, alpha_max=200.0, h_cap=50)
    n = int(o["n_accepted"][0])
    h = o["h_rec"][0, :n]
    assert o["n_rejected"][0] == 0 and o["status"][0] == 0
    np.testing.assert_array_equal(h[1:-1] / h[:-2], 200.0)
