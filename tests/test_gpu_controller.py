"""GPU vs oracle with the controller paths the default settings never take
(eq:controller in its PI form, reading c2; non-default safety and clamp
bounds, which take pow instead of the Newton root; a user first step), in
the forward solve and in the adjoint's checkpoint replay, which must
reproduce the PI memory ||e_prev|| stored in each checkpoint.

Parity bar as for the default controller: identical accepted and rejected
counts and every output within 1e-9 relative (floor 1) of the oracle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import gpu_solve, oracle_solve, rel_err, to_np  # noqa: E402
from parity_log import record  # noqa: E402
from paper_2609_28458_amd import api  # noqa: E402
from test_gpu_forward import CASES  # noqa: E402

TOL = 1e-9
NU = {"dopri5": 5, "tsit5": 5, "verner7": 7}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    api.lib()


def _controller(kind, tab):
    nu = NU[tab]
    if kind == "pi":          # PI form: beta1 = 0.7/nu, beta2 = 0.4/nu
        return dict(beta1=0.7 / nu, beta2=0.4 / nu)
    if kind == "wide_clamp":  # safety and bounds that rule out the Newton root
        return dict(safety=0.5, alpha_min=0.05, alpha_max=200.0)
    if kind == "pi_wide":     # both at once
        return dict(beta1=0.7 / nu, beta2=0.4 / nu, safety=0.8, alpha_min=0.1, alpha_max=10.0)
    return dict(h0=0.05)      # a user first step, default controller


def _parity(g, o, what):
    np.testing.assert_array_equal(g["n_accepted"], o["n_accepted"])
    np.testing.assert_array_equal(g["n_rejected"], o["n_rejected"])
    np.testing.assert_array_equal(g["status"], o["status"])
    e = float(rel_err(g["y_final"], o["y_final"]).max())
    if "y_out" in o:
        e = max(e, float(np.nanmax(rel_err(g["y_out"], o["y_out"]))))
    record(what, e, TOL)
    assert e <= TOL, e


@pytest.mark.parametrize("kind", ["pi", "wide_clamp", "pi_wide", "h0"])
@pytest.mark.parametrize("tab", ["dopri5", "tsit5", "verner7"])
@pytest.mark.parametrize("name,make", [CASES[0], CASES[2], CASES[3]],
                         ids=["harmonic", "loghalo", "spinprec"])
def test_controller_paths_match_oracle(orc, name, make, tab, kind):
    w = make(200)
    w["tableau"] = tab
    ctl = _controller(kind, tab)
    if kind == "h0" and name == "spinprec":
        ctl = dict(h0=1e-4)   # the precession variable v spans about 0.2
    if kind.startswith("pi") and name == "harmonic":
        # The starting-step rule can give Verner 7 on the oscillator at 1e-9 a
        # first step so short that its error norm (~1e-6) is pure rounding:
        # the I controller's factor is clamped at alpha_max there, PI's
        # (beta1 = 0.1) is not, so two correct codes that round differently
        # take next steps that differ by ~1e-4 and may end a step apart.  A
        # user first step near the tolerance's own step keeps every norm
        # above the rounding level.
        ctl = dict(ctl, h0=0.05)
    g = to_np(gpu_solve(w, api.Launch(**ctl)))
    o = oracle_solve(orc, w, **ctl)
    assert np.all(g["status"] == 0)
    _parity(g, o, f"controller {kind} {name} {tab}")
    # the variant really changes the steps (else the test would not test it)
    d = to_np(gpu_solve(w))
    assert not (np.array_equal(d["n_accepted"], g["n_accepted"])
                and np.array_equal(d["n_rejected"], g["n_rejected"])
                and np.array_equal(d["y_final"], g["y_final"]))


def test_pi_with_the_uneven_batch_and_groups(orc):
    """PI control on 16-lane groups and single lanes in one launch: bitwise
    equal to one lane per trajectory, and the oracle on a sample."""
    from paper_2609_28458_amd import inputs

    w = inputs.orbits_uneven(n=3000, seed=71)
    ctl = _controller("pi", "tsit5")
    order = np.argsort(-inputs.predicted_cost(w), kind="stable")
    a = to_np(gpu_solve(w, api.Launch(**ctl), order=order))
    b = to_np(gpu_solve(w, api.Launch(block=128, wide=300, **ctl), order=order))
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    idx = np.unique(np.concatenate([order[:40], np.arange(0, 3000, 97)]))
    o = oracle_solve(orc, w, idx, **ctl)
    np.testing.assert_array_equal(a["n_accepted"][idx], o["n_accepted"])
    np.testing.assert_array_equal(a["n_rejected"][idx], o["n_rejected"])
    e = float(rel_err(a["y_final"][:, idx], o["y_final"]).max())
    record("controller pi, uneven batch on groups", e, TOL)
    assert e <= TOL


def test_root_clamp_of_the_fast_controller(orc):
    """Norms far below 1e-15 (a state of size 1e-20 in a nearly free motion,
    omega = 1e-30): eq:controller gives safety * ||e||^(-1/7) >> alpha_max,
    so every step grows by alpha_max.  With safety 0.5 and alpha_max 100 the
    kernels' Newton root, whose input is clamped at 1e-30, would cap the
    factor at 0.5 * 1e15^(1/7) = 69.5; the host must route this controller
    through pow.  The GPU's step sizes are read off its store-mode tape."""
    y0 = np.array([[1e-20], [1e-20]])
    w = dict(rhs="harmonic", tableau="verner7", y0=y0, theta=np.array([1e-30]), t0=0.0,
             t1=1e9, rtol=1e-8, atol=1e-8)
    ctl = dict(safety=0.5, alpha_max=100.0, h0=1e-3)
    sol = gpu_solve(w, api.Launch(ckpt_every=1, ckpt_capacity=64, **ctl))
    g = to_np(sol)
    o = oracle_solve(orc, w, h_cap=64, **ctl)
    n = int(o["n_accepted"][0])
    h = o["h_rec"][0, :n]
    np.testing.assert_allclose(h[1:-1] / h[:-2], 100.0, rtol=1e-14)
    np.testing.assert_array_equal(g["n_accepted"], o["n_accepted"])
    # store-mode record j = (t_j, h_{j-1}, y_j), after the 256-byte counters
    tape = sol.workspace[256:256 + 64 * 4 * 8].view(torch.float64).reshape(64, 4).cpu().numpy()
    hg = tape[1:n + 1, 1]
    e = np.abs(hg - h) / h
    record("controller fast-root clamp (tiny norms): step sizes", e.max(), 1e-12)
    assert e.max() <= 1e-12, (hg, h)


@pytest.mark.parametrize("k", [1, 3], ids=["store", "ckpt3"])
@pytest.mark.parametrize("tab", ["dopri5", "verner7"])
def test_pi_adjoint_replays_the_controller_memory(orc, tab, k):
    """Adjoint of a PI-controlled solve: checkpoint mode replays each segment
    from (t, h, ||e_prev||, y, f) and must land on the next checkpoint bit for
    bit (no replay mismatch); the VJP equals cotangent . S of the oracle's
    forward sensitivities with the same controller."""
    name, make = CASES[2]
    w = make(150)
    w["tableau"] = tab
    ctl = _controller("pi_wide", tab)
    prob = api.make_problem(w["rhs"], tab, w["y0"], w["theta"], w["t0"], w["t1"], w["rtol"],
                            w["atol"], w["t_out"])
    d, n, K, p = prob.d, prob.n, prob.K, api.NPARAM[prob.rhs]
    sol = api.solve(prob, api.Launch(ckpt_every=k, ckpt_capacity=20000 if k == 1 else 4096,
                                     **ctl))
    torch.cuda.synchronize()
    assert bool((sol.status == 0).all())
    rng = np.random.default_rng(21)
    ybo = rng.normal(size=(1, d, K, n))
    ybf = rng.normal(size=(1, d, n))
    y0b, thb = api.solve_vjp(sol, ybar_final=ybf, ybar_out=ybo)
    torch.cuda.synchronize()
    assert sol.replay_mismatches() == 0
    th = np.repeat(np.asarray(w["theta"])[:, None], n, axis=1)
    o = oracle_solve(orc, {**w, "theta": th}, sens_cols=list(range(d + p)), **ctl)
    np.testing.assert_array_equal(sol.n_accepted.cpu().numpy(), o["n_accepted"])
    np.testing.assert_array_equal(sol.n_rejected.cpu().numpy(), o["n_rejected"])
    g = (np.einsum("jn,jcn->cn", ybf[0], o["S_final"])
         + np.einsum("jkn,jckn->cn", ybo[0], o["S_out"]))
    G = np.concatenate([y0b[0].cpu().numpy(), thb[0].cpu().numpy()])
    err = np.abs(G - g) / np.maximum(np.abs(g).max(axis=0), 1.0)
    record(f"vjp with PI control {tab} k={k}", err.max(), 1e-9)
    assert err.max() < 1e-9, err.max()
