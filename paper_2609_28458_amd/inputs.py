"""Seeded synthetic workloads (numpy only; no integrator arithmetic here).

Each generator returns a dict of float64 arrays in the structure-of-arrays
layouts of the C ABI ([d][n] states, [p] or [p][n] parameters, [K] or [K][n]
output nodes) plus the solver settings.  The same arrays feed the HIP path and
the CPU oracle.

The shapes follow the paper's three ensembles (Sections "Stellar streams",
"Dark energy", "Spin precession"); the exact draws are this project's synthetic
stand-ins for the paper's (unpublished) ensembles and data.
"""
from __future__ import annotations

import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def loghalo_ics(rng, n, v0, q, rc):
    """Orbits in the flattened logarithmic halo (eq:loghalo).

    Position (R cos phi, R sin phi, z) with R ~ U[0.5, 2], z ~ U[-0.3, 0.3],
    phi ~ U[0, 2 pi).  Speed = local circular speed v0 R / sqrt(R^2 + z^2/q^2
    + rc^2) times N(1, 0.1); direction tilted from the azimuthal unit vector by
    alpha ~ U[0, 0.3] rad towards cos(beta) R_hat + sin(beta) z_hat,
    beta ~ U[0, 2 pi).  v0, q, rc may be scalars or [n] arrays.
    """
    R = rng.uniform(0.5, 2.0, n)
    z = rng.uniform(-0.3, 0.3, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    vcirc = v0 * R / np.sqrt(R * R + z * z / (q * q) + rc * rc)
    speed = vcirc * rng.normal(1.0, 0.1, n)
    alpha = rng.uniform(0.0, 0.3, n)
    beta = rng.uniform(0.0, 2.0 * np.pi, n)
    Rhat = np.stack([np.cos(ph), np.sin(ph), np.zeros(n)])
    phat = np.stack([-np.sin(ph), np.cos(ph), np.zeros(n)])
    zhat = np.stack([np.zeros(n), np.zeros(n), np.ones(n)])
    dirv = np.cos(alpha) * phat + np.sin(alpha) * (np.cos(beta) * Rhat + np.sin(beta) * zhat)
    y0 = np.empty((6, n))
    y0[0] = R * np.cos(ph)
    y0[1] = R * np.sin(ph)
    y0[2] = z
    y0[3:] = speed * dirv
    return y0


def orbits_forward(n=1000, seed=1):
    """1,000 orbits, shared (v0, q, rc) = (1, 0.9, 0.1), t in [0, 50],
    Dopri5 at rtol 1e-8 / atol 1e-10, 64 output times 50 k / 64."""
    rng = _rng(seed)
    theta = np.array([1.0, 0.9, 0.1])
    y0 = loghalo_ics(rng, n, *theta)
    return dict(rhs="loghalo", tableau="dopri5", y0=y0, theta=theta, t0=0.0, t1=50.0,
                rtol=1e-8, atol=1e-10, t_out=50.0 * np.arange(1, 65) / 64.0)


def streams(n=1_000_000, seed=9, periods=3.7):
    """The paper's stream orbits (Section on streams): shared halo v_c = 1,
    R_c = 0.2, q = 0.7, orbits from near-circular to eccentric, in and out of
    the plane: R ~ U[0.5, 2], z ~ U[-0.3, 0.3], phi ~ U[0, 2 pi); speed =
    f v_circ(R, z), f ~ U[0.6, 1]; direction tilted from the azimuthal unit
    vector by alpha ~ U[0, pi/4] towards cos(beta) R_hat + sin(beta) z_hat,
    beta ~ U[0, 2 pi).  Each orbit runs for `periods` circular periods
    2 pi R / v_circ at its starting point; Tsit5 at rtol = atol = 3.16e-7;
    final state only.  The speed and tilt ranges are set so that the mean
    number of step attempts matches the paper's printed 171 (170.9 on the
    oracle).  Derivatives are taken with respect to (v_c, q): sensitivity
    columns 6 and 7."""
    rng = _rng(seed)
    v0, q, rc = 1.0, 0.7, 0.2
    R = rng.uniform(0.5, 2.0, n)
    z = rng.uniform(-0.3, 0.3, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    vcirc = v0 * R / np.sqrt(R * R + z * z / (q * q) + rc * rc)
    f = rng.uniform(0.6, 1.0, n)
    alpha = rng.uniform(0.0, 0.25 * np.pi, n)
    beta = rng.uniform(0.0, 2.0 * np.pi, n)
    Rhat = np.stack([np.cos(ph), np.sin(ph), np.zeros(n)])
    phat = np.stack([-np.sin(ph), np.cos(ph), np.zeros(n)])
    zhat = np.stack([np.zeros(n), np.zeros(n), np.ones(n)])
    dirv = np.cos(alpha) * phat + np.sin(alpha) * (np.cos(beta) * Rhat + np.sin(beta) * zhat)
    y0 = np.concatenate([np.stack([R * np.cos(ph), R * np.sin(ph), z]), f * vcirc * dirv])
    t1 = periods * 2.0 * np.pi * R / vcirc
    return dict(rhs="loghalo", tableau="tsit5", y0=y0, theta=np.array([v0, q, rc]), t0=0.0,
                t1=t1, rtol=3.16e-7, atol=3.16e-7, t_out=None, grad_cols=[6, 7])


def orbits_uneven(n=100_000, seed=2):
    """Uneven batch: per-orbit v0 ~ U[0.9, 1.1], q ~ U[0.7, 1], rc ~ U[0.05, 0.3],
    t_end ~ logU[10, 500], rtol ~ logU[1e-9, 1e-6] (atol = rtol), Tsit5,
    final state only."""
    rng = _rng(seed)
    v0 = rng.uniform(0.9, 1.1, n)
    q = rng.uniform(0.7, 1.0, n)
    rc = rng.uniform(0.05, 0.3, n)
    y0 = loghalo_ics(rng, n, v0, q, rc)
    t1 = np.exp(rng.uniform(np.log(10.0), np.log(500.0), n))
    rtol = np.exp(rng.uniform(np.log(1e-9), np.log(1e-6), n))
    return dict(rhs="loghalo", tableau="tsit5", y0=y0, theta=np.stack([v0, q, rc]),
                t0=0.0, t1=t1, rtol=rtol, atol=rtol.copy(), t_out=None)


def predicted_cost(w):
    """Heuristic cost of each trajectory for longest-first queue order: the
    number of dynamical times in the span times rtol^(-1/5) (a 5th-order
    method's steps per dynamical time).  For orbits in the logarithmic halo
    the dynamical time is (rc + r_E) / v0, with r_E the radius in the plane
    at which the potential equals the orbit's energy; otherwise the span
    itself stands in for it."""
    n = w["y0"].shape[1]
    span = np.broadcast_to(np.asarray(w["t1"], float) - np.asarray(w["t0"], float), (n,))
    rtol = np.broadcast_to(np.asarray(w["rtol"], float), span.shape)
    if w["rhs"] == "loghalo":
        th = np.asarray(w["theta"], float)
        th = th[:, None] if th.ndim == 1 else th
        v0, q, rc = (np.broadcast_to(th[i], (n,)) for i in range(3))
        y = w["y0"]
        Dn = rc * rc + y[0] ** 2 + y[1] ** 2 + y[2] ** 2 / (q * q)
        E = 0.5 * (y[3] ** 2 + y[4] ** 2 + y[5] ** 2) + 0.5 * v0 * v0 * np.log(Dn)
        r_E = np.sqrt(np.maximum(np.exp(2.0 * E / (v0 * v0)) - rc * rc, 0.0))
        span = span * v0 / (rc + r_E)
    return span * rtol ** (-0.2)


def orbits_gradient(n=100_000, seed=3):
    """As ``orbits_forward`` with t_end = 100, final state only, plus seeded
    targets T_i ~ N(0, 1)^3 for the loss sum_i |x_i(100) - T_i|^2."""
    w = orbits_forward(n, seed)
    rng = _rng(seed + 1000)
    w.update(t1=100.0, t_out=None, targets=rng.normal(0.0, 1.0, (3, n)))
    return w


def spin_precession(n=1_000_000, seed=4, n_grad=20_000):
    """Binaries: q ~ U[0.1, 1], chi1, chi2 ~ U[0, 1], isotropic unit spins,
    Lhat = z_hat; integrate in v = r^(-1/2) from r = 1000 to r = 10 with
    Verner 7 at rtol = atol = 3.16e-9; 32 nodes at r_k = 1000 * 10^(-2k/31)."""
    rng = _rng(seed)
    q = rng.uniform(0.1, 1.0, n)
    chi1 = rng.uniform(0.0, 1.0, n)
    chi2 = rng.uniform(0.0, 1.0, n)
    s1 = rng.normal(size=(3, n))
    s1 /= np.linalg.norm(s1, axis=0)
    s2 = rng.normal(size=(3, n))
    s2 /= np.linalg.norm(s2, axis=0)
    y0 = np.zeros((9, n))
    y0[2] = 1.0
    y0[3:6] = s1
    y0[6:9] = s2
    r_nodes = 1000.0 * 10.0 ** (-2.0 * np.arange(32) / 31.0)
    return dict(rhs="spinprec", tableau="verner7", y0=y0, theta=np.stack([q, chi1, chi2]),
                t0=1000.0 ** -0.5, t1=10.0 ** -0.5, rtol=3.16e-9, atol=3.16e-9,
                t_out=r_nodes ** -0.5, n_grad=n_grad)


def quintessence(n=10_000, seed=5, dense=False, omega_r=9.0e-5):
    """Thawing quintessence: lambda ~ U[0, 1.5], Omega_m ~ U[0.28, 0.34],
    Omega_r fixed; field at rest at z = 50; amplitude a0 = 1 - Omega_m -
    Omega_r (the frozen-field value); Dopri5 at rtol 1.78e-4, atol = 1e-3 rtol;
    nodes at 7 redshifts uniform in ln(1+z) on [0.3, 2.33] (dense variant: 64
    on [0, 2.5]), stored as N = -ln(1+z) in increasing order."""
    rng = _rng(seed)
    lam = rng.uniform(0.0, 1.5, n)
    om = rng.uniform(0.28, 0.34, n)
    orad = np.full(n, omega_r)
    a0 = 1.0 - om - orad
    if dense:
        z = np.expm1(np.linspace(np.log(3.5), 0.0, 64))
    else:
        z = np.expm1(np.linspace(np.log(3.33), np.log(1.3), 7))
    return dict(rhs="quint", tableau="dopri5", y0=np.zeros((3, n)),
                theta=np.stack([a0, lam, om, orad]), t0=-np.log(51.0), t1=0.0,
                rtol=1.78e-4, atol=1.78e-7, t_out=-np.log1p(z), z_nodes=z)


def de_profile_mocks(n_mocks=100, n_lambda=100, seed=6, omega_r=9.0e-5):
    """Synthetic coverage test of the dark-energy profile likelihood: a
    fiducial model (lambda 0.8, Omega_m 0.31, h = H0/H0_ref 1) observed through
    D_M and D_H at the 7 node redshifts of `quintessence`, n_mocks draws of
    1% Gaussian noise on each, the slope fixed on a grid of n_lambda values on
    [0, 1.5], and every minimisation started at Omega_m 0.30, h 1 and the
    frozen-field amplitude.  Minimisation i uses mock i // n_lambda and slope
    lam_grid[i % n_lambda].  Only the draws live here: the data are
    D_fid (1 + rel_noise * eps), D_fid from whichever solver runs the fit.
    N_spline holds the 64 dense nodes of `quintessence` through which the
    profile's spline reads the model at the data redshifts."""
    rng = _rng(seed)
    q = quintessence(n=1, omega_r=omega_r)
    qd = quintessence(n=1, dense=True, omega_r=omega_r)
    return dict(lam_grid=np.linspace(0.0, 1.5, n_lambda), eps=rng.normal(size=(n_mocks, 2, 7)),
                rel_noise=0.01, fid=dict(lam=0.8, om=0.31, h=1.0), start=dict(om=0.30, h=1.0),
                omega_r=omega_r, N_nodes=q["t_out"], z_nodes=q["z_nodes"],
                N_spline=qd["t_out"], t0=q["t0"],
                tableau="dopri5", rtol=q["rtol"], atol=q["atol"], iters=20, newton=3,
                mu=1e-3, trust=(0.05, 0.05))


def _logu(rng, lo, hi, n):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n))


# Nominal rates of the eight-species network (k1..k10, source s, k12).
KIN8_NOMINAL = np.array([1.0, 0.5, 10.0, 0.1, 5.0, 3.0e3, 100.0, 1.0, 100.0, 0.01, 1.0e-3, 1.0])


def kinetics3(n=100_000, seed=7, K=16):
    """Stiff three-species autocatalytic kinetics (a -> b, b + c -> 2c,
    c -> a), a stand-in for the classic stiff chemistry problems: rates
    k1 ~ logU[1e-2, 1e-1], k2 ~ logU[1e6, 1e7], k3 ~ logU[0.1, 1], so the fast
    and slow time-scales differ by 7-9 decades; start (1 - c0, 0, c0),
    c0 ~ logU[1e-4, 1e-2]; spans t1 ~ logU[10, 1e4]; Rodas4 at rtol 1e-6,
    atol 1e-10; K output times per trajectory, log-spaced from t1 1e-6 to t1."""
    rng = _rng(seed)
    k = np.stack([_logu(rng, 1e-2, 1e-1, n), _logu(rng, 1e6, 1e7, n), _logu(rng, 0.1, 1.0, n)])
    c0 = _logu(rng, 1e-4, 1e-2, n)
    y0 = np.stack([1.0 - c0, np.zeros(n), c0])
    t1 = _logu(rng, 10.0, 1e4, n)
    t_out = t1[None, :] * np.logspace(-6, 0, K)[:, None] if K else None
    return dict(rhs="kin3", tableau="rodas4", y0=y0, theta=k, t0=0.0, t1=t1, rtol=1e-6,
                atol=1e-10, t_out=t_out)


def kinetics8(n=100_000, seed=8, K=16):
    """Stiff eight-species network with one reversible bilinear step (see the
    kin8 right-hand side): every rate its nominal value (KIN8_NOMINAL) times
    logU[1/3, 3], so the time-scales span about five decades; start y1 = 1,
    y5 = 1e-3, the rest 0; spans t1 ~ logU[100, 1000]; Rodas4 at rtol 1e-6,
    atol 1e-10; K output times log-spaced from t1 1e-6 to t1."""
    rng = _rng(seed)
    k = KIN8_NOMINAL[:, None] * _logu(rng, 1.0 / 3.0, 3.0, 12 * n).reshape(12, n)
    y0 = np.zeros((8, n))
    y0[0] = 1.0
    y0[4] = 1e-3
    t1 = _logu(rng, 100.0, 1000.0, n)
    t_out = t1[None, :] * np.logspace(-6, 0, K)[:, None] if K else None
    return dict(rhs="kin8", tableau="rodas4", y0=y0, theta=k, t0=0.0, t1=t1, rtol=1e-6,
                atol=1e-10, t_out=t_out)


# Nominal rate constants of the two classic stiff chemistry problems.
ROBER_NOMINAL = np.array([0.04, 3.0e7, 1.0e4])
HIRES_NOMINAL = np.array([1.71, 0.43, 8.32, 0.0007, 0.035, 1.12, 280.0, 0.69])
HIRES_Y0 = np.array([1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0057])
HIRES_T1 = 321.8122


def robertson(n=100_000, seed=10, K=16, spread=2.0):
    """Robertson's reaction (rober right-hand side): each rate its nominal
    value (0.04, 3e7, 1e4) times logU[1/spread, spread]; start (1, 0, 0);
    spans t1 ~ logU[40, 4e5] (the textbook interval is [0, 40], its long-time
    variants reach 1e11); Rodas4 at rtol 1e-6, atol 1e-10 (y2 stays below
    4e-5); K output times log-spaced from t1 1e-6 to t1.  spread = 1 gives
    the textbook problem for every trajectory."""
    rng = _rng(seed)
    k = ROBER_NOMINAL[:, None] * _logu(rng, 1.0 / spread, spread, 3 * n).reshape(3, n)
    y0 = np.zeros((3, n))
    y0[0] = 1.0
    t1 = _logu(rng, 40.0, 4.0e5, n)
    t_out = t1[None, :] * np.logspace(-6, 0, K)[:, None] if K else None
    return dict(rhs="rober", tableau="rodas4", y0=y0, theta=k, t0=0.0, t1=t1, rtol=1e-6,
                atol=1e-10, t_out=t_out)


def hires(n=100_000, seed=11, K=16, spread=1.25):
    """HIRES, the plant-physiology problem (hires right-hand side): each of
    its eight independent constants its nominal value times
    logU[1/spread, spread]; the textbook start (1, 0, 0, 0, 0, 0, 0, 0.0057)
    and span [0, 321.8122]; Rodas4 at rtol 1e-6, atol 1e-10; K output times
    uniform in (0, t1].  spread = 1 gives the textbook problem."""
    rng = _rng(seed)
    k = HIRES_NOMINAL[:, None] * _logu(rng, 1.0 / spread, spread, 8 * n).reshape(8, n)
    y0 = np.repeat(HIRES_Y0[:, None], n, axis=1)
    t_out = np.linspace(HIRES_T1 / K, HIRES_T1, K) if K else None
    return dict(rhs="hires", tableau="rodas4", y0=y0, theta=k, t0=0.0, t1=HIRES_T1, rtol=1e-6,
                atol=1e-10, t_out=t_out)
