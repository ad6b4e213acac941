"""Benchmark: ensemble solves and their gradients on one MI355X, at fixed error.

Headline (N = 1): 10^6 spin-precession binaries (orbit-averaged 2PN
precession of L, S1, S2 in v = r^(-1/2) from r = 1000 to 10, q ~ U[0.1, 1],
chi1, chi2 ~ U[0, 1], isotropic spins), Verner 7, 32 outputs, at rtol = atol
= 1e-11: the loosest tolerance on the paper's quarter-decade grid that meets
the 2e-7 rad precession budget from r = 1000 (the configured 3.16e-9 does
not, and is reported beside it, labelled so).  One step is one complete
ensemble solve from device-resident inputs: the longest-first queue order
built on the device from the pilot-fitted cost (counting sort), the persistent
solve kernel, and the outputs' shortened steps, captured once in one graph and
replayed.  `value` is solves per second.  The pilot solve and fit that give
the cost model are timed and reported next to it (with a value that includes
them).  The 99th-percentile angle error against a tight reference is printed
beside the timing.

Also reported: the other configurations, each with its accuracy column
(eq:accept budgets against tight references):
  * c2: 100,000 uneven orbits (Tsit5, per-orbit rtol and t_end), order built
    on the device inside the graph; roofline and critical path;
  * c1: 1,000 orbits with 64 outputs (latency), and the same recipe at 10^6;
  * c3: the gradient workload (grad/forward time ratio, adjoint roofline and
    critical path);
  * c5: 10^4 cosmologies (7 and 64 redshifts), and the dark-energy profile;
  * the stiff path on its four problems; precession gradients;
  * cpu_baseline: the CPU oracle on a bounded sample of the headline
    workload, all host cores and one core.

Modes: `--mode profile` runs the headline graph only (for rocprofv3 kernel
traces of exactly the timed launch); `--mode traffic` runs a device copy of
known size and one headline solve (for FETCH_SIZE / WRITE_SIZE passes);
`--mode lone` solves the headline's longest binary alone.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_VECTOR_TFLOPS = 78.6   # MI355X: 256 CU x 2.4 GHz x 128 FP64 flop/clk
# Algorithmic FP64 flops of one step attempt (fma = 2, div / sqrt / root / reciprocal = 1):
#   stage sums 2 d (nnz(A) + s - 1), the update of a non-FSAL pair 2 d (nnz(b) + 1),
#   stage times 2 (s - 1), error weights 2 d nnz(b - bhat) + d, norm 5 d + 2, controller
#   and clipping 5, and one right-hand side per new stage (s - 1 for FSAL pairs, s else).
#   Tsit5 + log halo (d 6, nnz(A) 21, nnz(e) 7, 13 per evaluation): 324 + 12 + 90 + 32 + 5
#   + 78 = 541.  Dopri5 + log halo (nnz(A) 20, nnz(e) 6): 312 + 12 + 78 + 32 + 5 + 78 = 517.
#   Verner 7 + precession (d 9, s 10, nnz(A) 36, nnz(b) 7, nnz(e) 8, 119 per evaluation of
#   the unfolded right-hand side, the form the adjoint differentiates; the solve's folded
#   form issues 97): 810 + 144 + 18 + 153 + 47 + 5 + 1190 = 2367; one output node (a
#   shortened step) adds 9 evaluations and the stage sums and update, 1071 + 810 + 144 = 2025.
FLOPS_PER_ATTEMPT = {("tsit5", "loghalo"): 541, ("dopri5", "loghalo"): 517,
                     ("verner7", "spinprec"): 2367}
FLOPS_PER_NODE = {("verner7", "spinprec"): 2025, ("dopri5", "loghalo"): 168}
# Reverse of one accepted step (store-mode tape, one loss): recompute the first
# right-hand side, the stage points and right-hand sides of the stages that feed
# the step, then seed h b_j lam, reverse every feeding stage through the
# right-hand side's VJP (46 flops for the log halo) and the transposed stage sums.
FLOPS_PER_VJP_STEP = {("dopri5", "loghalo"): 880}
HEADLINE_RTOL = 1e-11
PREC_BUDGET_RAD = 2e-7        # eq:prec-err
ORBIT_BUDGET = 1e-4           # eq:st-fwderr
DE_BUDGET = 1e-4              # distances, c/H0
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles",
                               "traffic_solve_kernel_verner7_spinprec_1m_binaries_rtol1e-11.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2609_28458_amd", "csrc", f)
                  for f in ("gs_kernels.hpp", "gs_rhs.hpp", "gs_tableaux.hpp")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1_000_000, help="binaries of the headline")
    ap.add_argument("--mode", choices=("full", "profile", "traffic", "lone", "gradient"),
                    default="full")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-rest", action="store_true", help="headline only")
    return ap.parse_args()


def timed(fn, steps, warmup, torch):
    """ms per call of fn: warmup calls, then `steps` calls between two HIP
    events on the current stream."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


def wall_ms(fn, torch):
    torch.cuda.synchronize()
    t = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) * 1e3, out


def p99(x):
    return float(np.quantile(np.asarray(x), 0.99))


def mk(api, w, **over):
    w = {**w, **over}
    return api.make_problem(w["rhs"], w["tableau"], w["y0"], w["theta"], w["t0"], w["t1"],
                            w["rtol"], w["atol"], w.get("t_out"))


def subset(w, idx):
    """The trajectories idx of a workload dict (per-trajectory arrays sliced)."""
    n = w["y0"].shape[1]
    out = {}
    for k, v in w.items():
        if isinstance(v, np.ndarray) and v.shape[-1:] == (n,):
            out[k] = v[..., idx]
        else:
            out[k] = v
    return out


# ---- accuracy measures of eq:accept ------------------------------------------------------

def angle_error(a, b):
    """eq:prec-err: the largest angle between the L, S1, S2 of two states [9][m]."""
    eps = np.zeros(a.shape[1])
    for s in range(3):
        x, y = a[3 * s:3 * s + 3], b[3 * s:3 * s + 3]
        ang = np.arctan2(np.linalg.norm(np.cross(x, y, axis=0), axis=0), np.sum(x * y, axis=0))
        eps = np.maximum(eps, ang)
    return eps


def orbit_scales(y0, theta):
    """r_E and v_E of each orbit (eq:st-scales) from its energy."""
    th = np.asarray(theta, float)
    th = th[:, None] if th.ndim == 1 else th
    v0, q, rc = th
    Dn = rc * rc + y0[0] ** 2 + y0[1] ** 2 + y0[2] ** 2 / q ** 2
    E = 0.5 * (y0[3] ** 2 + y0[4] ** 2 + y0[5] ** 2) + 0.5 * v0 * v0 * np.log(Dn)
    return np.sqrt(np.exp(2 * E / v0 ** 2) - rc * rc), np.sqrt(2 * E - v0 * v0 * np.log(rc * rc))


def orbit_error(y, ref, y0, theta):
    """eq:st-fwderr: max(|dx| / r_E, |dv| / v_E) per orbit; y, ref [6][...][m]."""
    rE, vE = orbit_scales(y0, theta)
    dx = np.linalg.norm(y[:3] - ref[:3], axis=0) / rE
    dv = np.linalg.norm(y[3:] - ref[3:], axis=0) / vE
    e = np.maximum(dx, dv)
    return e.max(axis=0) if e.ndim == 2 else e


def accuracy_row(eps, budget, what, ref):
    eps = np.asarray(eps)
    return {"measure": what, "p99": p99(eps), "max": float(eps.max()), "budget": budget,
            "over_budget": int(np.sum(eps > budget)), "sample": int(eps.size), "reference": ref}


# ---- the headline: 10^6 binaries at fixed error --------------------------------------------

def spin_features(torch, prob):
    """Features of the pilot cost model of a precession ensemble, on the device:
    log q, both spin magnitudes, and the cosines between L, S1 and S2."""
    y, th = prob.y0, prob.theta
    return torch.stack([torch.log(th[0]), th[1], th[2], (y[0:3] * y[3:6]).sum(0),
                        (y[0:3] * y[6:9]).sum(0), (y[3:6] * y[6:9]).sum(0)])


def headline(args, torch, api, inputs, autotune):
    w = inputs.spin_precession(n=args.n)
    w.update(rtol=HEADLINE_RTOL, atol=HEADLINE_RTOL)
    n = w["y0"].shape[1]
    prob = mk(api, w)
    # The cost model: a pilot solve of 4,096 binaries over the last decade of the
    # separation only (r = 100 -> 10, where the precession is fastest: about 2,000
    # attempts instead of 65,000, and the pilot takes as long as its longest binary),
    # a least-squares fit of their attempts on the features, evaluated for every
    # binary (set-up of the order; timed and reported).  Its rank correlation with the
    # full solve's attempts is 0.98, as good as a pilot over the whole span.
    pilot = mk(api, w, t0=100.0 ** -0.5, t_out=None)
    # The pilot's 4,096 binaries fill 64 of the 1,024 SIMDs at one lane each; on 16-lane
    # groups (the same steps, bit for bit) they spread over the chip.
    # The first call also pays one-time costs of the process (loading the kernels' code,
    # the host solver's set-up); the pilot as a repeated step of building the order is
    # the second call.  Both are reported.
    plaunch = api.Launch(wide=4096)
    pilot_first_ms, cost = wall_ms(
        lambda: autotune.pilot_cost(pilot, spin_features(torch, pilot), launch=plaunch), torch)
    pilot_ms, cost = wall_ms(
        lambda: autotune.pilot_cost(pilot, spin_features(torch, pilot), launch=plaunch), torch)
    args.pilot_first_ms = pilot_first_ms
    cost = cost.contiguous()
    # Launch: 256-lane workgroups, the occupancy-limited grid (one wave per SIMD), and a
    # wavefront refills as soon as one lane is idle (65,000 attempts per binary make the
    # refill's own cost negligible; waiting for 8 idle lanes measured 3.8% slower).
    sol = api.Solution(prob, api.Launch(refill=1))
    sol.queue_order(cost)  # order and its workspace exist before the capture
    torch.cuda.synchronize()

    def body(stream):
        sol.queue_order(cost, stream=stream)
        sol.run(stream=stream)

    graph = api.Captured(body)
    return w, prob, sol, graph, cost, pilot_ms


def headline_rows(args, torch, api, inputs, autotune, w, prob, sol, graph, cost, pilot_ms):
    n = prob.n
    ms = timed(graph.launch, args.steps, args.warmup, torch)
    nacc = int(sol.n_accepted.to(torch.int64).sum())
    att_each = (sol.n_accepted + sol.n_rejected).to(torch.int64)
    attempts = int(att_each.sum())
    max_att = int(att_each.max())
    ok = bool((sol.status == 0).all())
    fpa = FLOPS_PER_ATTEMPT[("verner7", "spinprec")]
    fpn = FLOPS_PER_NODE[("verner7", "spinprec")]
    log(f"[bench] headline: {n} binaries at {HEADLINE_RTOL:g}: {ms:.1f} ms per solve, "
        f"{attempts} attempts, all ok {ok}; pilot {pilot_ms:.1f} ms")

    # Accuracy: final spin and orbital directions against Verner 7 at 1e-13 on
    # 20,000 random binaries (eq:prec-err, budget 2e-7 rad).
    idx = np.sort(np.random.default_rng(17).choice(n, min(n, 20_000), replace=False))
    ws = subset(w, idx)
    ref = api.solve(mk(api, ws, rtol=1e-13, atol=1e-13, t_out=None))
    torch.cuda.synchronize()
    yf = sol.y_final.cpu().numpy()
    eps = angle_error(yf[:, idx], ref.y_final.cpu().numpy())
    acc = accuracy_row(eps, PREC_BUDGET_RAD, "eq:prec-err, final L, S1, S2 (rad)",
                       "Verner 7 at rtol = atol = 1e-13 on the GPU (parity-tested against "
                       "the oracle)")
    log(f"[bench] headline accuracy: P99 {acc['p99']:.3e} rad, {acc['over_budget']} of "
        f"{acc['sample']} over 2e-7")

    # Kernel time with HIP events on the launch stream (a direct gs_solve: queue reset,
    # status fill for the given order, the solve kernel, the outputs' shortened steps).
    s = torch.cuda.current_stream()

    def direct():
        sol.args.stream = s.cuda_stream
        api.gs_solve(sol.args)

    ms_kernel = timed(direct, 2, 0, torch)
    achieved = attempts * fpa / (ms_kernel * 1e-3) / 1e12
    # Its critical path: the longest binary alone on one lane.
    i_long = int(torch.argmax(att_each))
    one = subset(w, [i_long])
    lsol = api.Solution(mk(api, one), api.Launch(block=64))
    ms_lone = timed(lambda: lsol.run(), 1, 1, torch)
    traffic, traffic_src = committed_traffic()
    roofline = {
        "bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_VECTOR_TFLOPS,
        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_VECTOR_TFLOPS, 4),
        "traffic": traffic, "traffic_source": traffic_src,
        "kernel": "gs::solve_kernel<Verner7, SpinPrec, true, false>",
        "flops_per_attempt": fpa, "attempts_per_launch": attempts,
        "ms_per_launch": round(ms_kernel, 3),
        "ms_per_launch_covers": "queue reset, status fill, solve kernel and the 32e6 "
                                "shortened-step outputs (a separate kernel, ~0.1% of it); "
                                "only the solve kernel's flops are counted",
        "output_flops_not_counted": n * prob.K * fpn,
        "critical_path": {"max_attempts_one_binary": max_att,
                          "longest_binary_alone_ms": round(ms_lone, 1),
                          "batch_over_longest_alone": round(ms_kernel / ms_lone, 3)}}
    log(f"[bench] headline kernel {ms_kernel:.1f} ms = {achieved:.2f} TFLOP/s "
        f"({achieved / PEAK_FP64_VECTOR_TFLOPS:.1%}); longest binary alone {ms_lone:.1f} ms")
    out = {
        "metric": "solves/s + accepted RK steps/s at fixed error; grad/forward time ratio",
        "value": n / (ms * 1e-3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "spin_precession_1m_r1000_to_10_verner7_rtol1e-11_32_outputs",
                   "n": n, "rhs": "spinprec (orbit-averaged 2PN precession)",
                   "tableau": "verner7", "rtol": HEADLINE_RTOL, "atol": HEADLINE_RTOL,
                   "K": prob.K, "r": "1000 -> 10",
                   "step": "one graph: longest-first order built on the device from the "
                           "pilot-fitted cost (counting sort), persistent solve, shortened-"
                           "step outputs"},
        "accuracy": acc,
        "accepted_steps_per_s": nacc / (ms * 1e-3),
        "attempts_per_s": attempts / (ms * 1e-3),
        "mean_attempts": attempts / n,
        "all_trajectories_ok": ok,
        "order_setup": {"what": "pilot solve of 4,096 binaries from r = 100 to 10 on 16-lane "
                                "groups (no "
                                "outputs), least-squares fit of their attempts on log q, chi1, "
                                "chi2 and the three cosines, fitted cost of all binaries",
                        "ms": round(pilot_ms, 1),
                        "ms_first_call_of_the_process": round(getattr(args, "pilot_first_ms",
                                                                      pilot_ms), 1),
                        "value_including_setup": n / ((ms + pilot_ms) * 1e-3)},
        "roofline": roofline,
    }
    # The configured tolerance, 3.16e-9: it misses the precession budget from r = 1000.
    w9 = {**w, "rtol": 3.16e-9, "atol": 3.16e-9}
    p9 = mk(api, w9)
    s9 = api.Solution(p9, api.Launch(refill=1))
    s9.queue_order(cost)
    ms9 = timed(lambda: (s9.queue_order(cost), s9.run()), 1, 1, torch)
    e9 = angle_error(s9.y_final.cpu().numpy()[:, idx], ref.y_final.cpu().numpy())
    att9 = int((s9.n_accepted + s9.n_rejected).to(torch.int64).sum())
    out["configured_tolerance_misses_budget"] = {
        "rtol": 3.16e-9, "ms": round(ms9, 1), "solves_per_s": n / (ms9 * 1e-3),
        "attempts": att9,
        "frac": round(att9 * fpa / (ms9 * 1e-3) / 1e12 / PEAK_FP64_VECTOR_TFLOPS, 4),
        "accuracy": accuracy_row(e9, PREC_BUDGET_RAD, "eq:prec-err (rad)", "as above"),
        "label": "misses the 2e-7 rad budget from r = 1000"}
    log(f"[bench] configured 3.16e-9: {ms9:.1f} ms, P99 {p99(e9):.3e} rad (misses budget)")
    del s9, lsol, ref
    return out, ms


def committed_traffic():
    """HBM bytes per launch from the committed PMC summary, if it was taken
    on the current kernel source; else None."""
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None, "no PMC summary"
    m = re.search(r"kernel source sha: (\w+)", text)
    b = re.search(r"HBM bytes per launch: ([0-9.eE+]+)", text)
    if not m or not b:
        return None, "summary unreadable"
    if m.group(1) != kernel_source_sha():
        return None, "kernel changed since the counters were taken"
    return float(b.group(1)), "committed rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated"


# ---- c2: 100,000 uneven orbits ---------------------------------------------------------

def c2_uneven(args, torch, api, inputs, autotune):
    w = inputs.orbits_uneven()
    prob = mk(api, w)
    n = prob.n
    base = api.Solution(prob, api.Launch())
    order = base.queue_order().clone()
    torch.cuda.synchronize()
    launch = autotune.tune_forward(prob, order=order, use_cache=False)
    sol = api.Solution(prob, launch)
    sol.queue_order()

    def body(stream):
        sol.queue_order(stream=stream)
        sol.run(stream=stream)

    graph = api.Captured(body)
    ms = timed(graph.launch, 20, 3, torch)
    ms_order = timed(lambda: base.queue_order(), 20, 3, torch)
    att_each = (sol.n_accepted + sol.n_rejected).to(torch.int64)
    attempts, max_att = int(att_each.sum()), int(att_each.max())
    nacc = int(sol.n_accepted.to(torch.int64).sum())
    s = torch.cuda.current_stream()

    def direct():
        sol.args.stream = s.cuda_stream
        api.gs_solve(sol.args)

    ms_kernel = timed(direct, 20, 1, torch)
    fpa = FLOPS_PER_ATTEMPT[("tsit5", "loghalo")]
    achieved = attempts * fpa / (ms_kernel * 1e-3) / 1e12
    i_long = int(torch.argmax(att_each))
    lprob = mk(api, subset(w, [i_long]))
    ms_lone = timed(lambda: api.solve(lprob, api.Launch(block=64)), 3, 1, torch)
    ms_group = timed(lambda: api.solve(lprob, api.Launch(block=64, wide=1)), 3, 1, torch)
    # accuracy: final states of 10,000 orbits against Verner 7 at 1e-13
    idx = np.sort(np.random.default_rng(18).choice(n, 10_000, replace=False))
    ws = subset(w, idx)
    ref = api.solve(mk(api, ws, tableau="verner7", rtol=1e-13, atol=1e-13))
    torch.cuda.synchronize()
    eps = orbit_error(sol.y_final.cpu().numpy()[:, idx], ref.y_final.cpu().numpy(), ws["y0"],
                      ws["theta"])
    # the two other arms: static one lane per trajectory, eight cost buckets
    st = api.Solution(prob, api.Launch(schedule="static", block=256))
    ms_static = timed(lambda: st.run(), 5, 1, torch)
    cost = inputs.predicted_cost(w)
    qs = np.quantile(cost, np.linspace(0, 1, 9))
    bsols = []
    for b in range(8):
        sel = np.nonzero((cost >= qs[b]) & ((cost < qs[b + 1]) if b < 7 else True))[0]
        bsols.append(api.Solution(mk(api, subset(w, sel)), api.Launch(schedule="static",
                                                                      block=256)))

    def buckets():
        for bs in bsols:
            bs.run()

    ms_buckets = timed(buckets, 5, 1, torch)
    res = {"workload": "100,000 orbits, per-orbit (v0, q, rc), t_end ~ logU[10, 500], "
                       "rtol ~ logU[1e-9, 1e-6], atol = rtol, Tsit5, final states",
           "ms": round(ms, 4), "solves_per_s": n / (ms * 1e-3),
           "accepted_steps_per_s": nacc / (ms * 1e-3), "attempts_per_s": attempts / (ms * 1e-3),
           "step": "one graph: device order (dynamical-time cost model, counting sort) and "
                   "the persistent solve", "ms_order_build": round(ms_order, 4),
           "launch": {k: launch.__dict__[k] for k in ("block", "grid", "refill", "wide")},
           "accuracy": accuracy_row(eps, ORBIT_BUDGET, "eq:st-fwderr, final state",
                                    "Verner 7 at 1e-13 on the GPU, 10,000 orbits"),
           "roofline": {"bound": "alu", "kernel": "gs::solve_kernel<Tsit5, LogHalo>",
                        "flops_per_attempt": fpa, "attempts": attempts,
                        "ms_per_launch": round(ms_kernel, 4), "achieved": round(achieved, 3),
                        "frac": round(achieved / PEAK_FP64_VECTOR_TFLOPS, 4),
                        "critical_path": {"max_attempts": max_att,
                                          "longest_alone_ms": {"one_lane": round(ms_lone, 3),
                                                               "group": round(ms_group, 3)},
                                          "batch_over_longest_alone":
                                              round(ms_kernel / min(ms_lone, ms_group), 3)}},
           "arms_ms": {"persistent_graph": round(ms, 4), "static_one_lane_each":
                       round(ms_static, 4), "eight_cost_buckets": round(ms_buckets, 4)},
           "all_ok": bool((sol.status == 0).all())}
    log(f"[bench] c2: {ms:.3f} ms ({n / ms * 1e3:.3e} solves/s), order build {ms_order:.4f} ms, "
        f"P99 {p99(eps):.2e}; static {ms_static:.2f}, buckets {ms_buckets:.2f}")
    return res


# ---- c1: 1,000 orbits, 64 outputs; and the recipe at 10^6 ------------------------------------

def c1_forward(torch, api, inputs, autotune):
    w = inputs.orbits_forward()
    prob = mk(api, w)
    # one lane per orbit (16 wavefronts), and every orbit on a 16-lane group
    # (250 wavefronts, one state component per lane), each captured in a graph
    ms_by = {}
    for name, L in (("lanes", api.Launch()), ("groups", api.Launch(wide=prob.n))):
        sol = api.Solution(prob, L)
        graph = api.Graph(sol)
        ms_by[name] = round(timed(lambda: graph.launch(), 20, 3, torch), 4)
        graph.close()
    ms = min(ms_by.values())
    ref = api.solve(mk(api, w, tableau="verner7", rtol=1e-13, atol=1e-13))
    torch.cuda.synchronize()
    eps = orbit_error(sol.y_out.cpu().numpy(), ref.y_out.cpu().numpy(), w["y0"], w["theta"])
    res = {"workload": "1,000 orbits, shared halo (1, 0.9, 0.1), Dopri5 1e-8 / 1e-10, 64 "
                       "outputs to t = 50", "ms": ms, "ms_by_mapping": ms_by,
           "solves_per_s": prob.n / (ms * 1e-3),
           "accuracy": accuracy_row(eps, ORBIT_BUDGET, "eq:st-fwderr over the 64 outputs",
                                    "Verner 7 at 1e-13 on the GPU"),
           "note": "latency-bound: one lane per orbit is 16 wavefronts on 1,024 SIMDs; "
                   "groups put one state component per lane"}
    log(f"[bench] c1: {ms:.3f} ms ({ms_by}), P99 {p99(eps):.2e}")
    # the same recipe at 10^6 orbits, outputs [K][n][d] and [d][K][n]
    nc = 1_000_000
    cw = inputs.orbits_forward(n=nc, seed=1)
    cprob = mk(api, cw)
    tmp = api.Solution(cprob, api.Launch())
    corder = tmp.queue_order().clone()
    del tmp
    claunch = autotune.tune_forward(cprob, order=corder, use_cache=False)
    csol = api.Solution(cprob, claunch)
    csol.set_order(corder)
    ms_dkn = timed(lambda: csol.run(), 3, 1, torch)
    att_c = int((csol.n_accepted + csol.n_rejected).to(torch.int64).sum())
    del csol
    csol = api.Solution(cprob, api.Launch(**{**claunch.__dict__, "out_layout": "knd"}))
    csol.set_order(corder)
    ms_c = timed(lambda: csol.run(), 3, 1, torch)
    fl_c = (att_c * FLOPS_PER_ATTEMPT[("dopri5", "loghalo")]
            + nc * cprob.K * FLOPS_PER_NODE[("dopri5", "loghalo")])
    ach_c = fl_c / (min(ms_c, ms_dkn) * 1e-3) / 1e12
    res["at_1m"] = {"workload": "the same recipe at 1,000,000 orbits, longest first",
                    "ms_out_layout_knd": round(ms_c, 3), "ms_out_layout_dkn": round(ms_dkn, 3),
                    "attempts": att_c, "achieved": round(ach_c, 3), "unit": "TFLOP/s",
                    "frac": round(ach_c / PEAK_FP64_VECTOR_TFLOPS, 4),
                    "all_ok": bool((csol.status == 0).all())}
    log(f"[bench] c1 at 10^6: [K][n][d] {ms_c:.3f} ms, [d][K][n] {ms_dkn:.3f} ms "
        f"({ach_c / PEAK_FP64_VECTOR_TFLOPS:.1%} at the faster)")
    del csol
    return res


# ---- c3: the gradient workload -------------------------------------------------------------

def c3_gradient(torch, api, inputs, autotune):
    wg = inputs.orbits_gradient()
    pg = mk(api, wg)
    n = pg.n
    reps = 5
    T = torch.as_tensor(wg["targets"], device="cuda")
    tmp = api.Solution(pg, api.Launch())
    gorder = tmp.queue_order().clone()
    del tmp
    flaunch = autotune.tune_forward(pg, order=gorder, use_cache=False)
    plain = api.Solution(pg, flaunch)
    plain.set_order(gorder)
    ms_fwd = timed(lambda: plain.run(), reps, 1, torch)
    nmax = int(plain.n_accepted.max())
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    ybf = torch.zeros((1, 6, n), dtype=torch.float64, device="cuda")

    def grad_ms(block, grid, k, order, wide=0, adj=None):
        """One gradient step: forward with tape (block, grid, wide), then the adjoint
        (on the same shape, or on adj = (block, grid, wide)); the adjoint's groups
        need the store-mode tape (k = 1)."""
        ab, ag, aw = adj or (block, grid, wide)
        aw = aw if k == 1 else 0
        taped = api.Solution(pg, api.Launch(block=block, grid=grid, ckpt_every=k,
                                            ckpt_capacity=nmax // k + 2, wide=wide))
        if order is not None:
            taped.set_order(order)

        def grad_step():
            taped.run()
            ybf[0, :3] = 2.0 * (taped.y_final[:3] - T)
            api.solve_vjp(taped, ybar_final=ybf, block=ab, grid=ag, wide=aw)

        return timed(grad_step, reps, 1, torch)

    shapes = {"block 256, occupancy grid, longest first": (256, 0, gorder, 0),
              "block 128, 2 waves per CU, longest first": (128, 2 * cus, gorder, 0),
              "block 64, 1 wave per SIMD, longest first": (64, 4 * cus, gorder, 0),
              "block 256, 1 wave per SIMD, longest first": (256, cus, gorder, 0),
              "block 128, 2 waves per CU, longest first, 256 on groups":
                  (128, 2 * cus, gorder, 256),
              "block 64, 1 wave per SIMD, longest first, 256 on groups":
                  (64, 4 * cus, gorder, 256)}
    by_shape = {name: round(grad_ms(sh[0], sh[1], 1, sh[2], sh[3]), 4)
                for name, sh in shapes.items()}
    # The two passes are separate launches, so each can take its own shape: the
    # forward with tape and the adjoint timed alone over the same shapes, then the
    # gradient step with the fastest of each.
    fwd_alone, adj_alone = {}, {}
    for name, (b, g, o, wd) in shapes.items():
        t1 = api.Solution(pg, api.Launch(block=b, grid=g, ckpt_every=1, ckpt_capacity=nmax + 2,
                                         wide=wd))
        t1.set_order(o)
        fwd_alone[name] = round(timed(lambda: t1.run(), reps, 1, torch), 4)
        ybf[0, :3] = 2.0 * (t1.y_final[:3] - T)
        adj_alone[name] = round(timed(lambda: api.solve_vjp(t1, ybar_final=ybf, block=b,
                                                            grid=g, wide=wd), reps, 1, torch), 4)
        del t1
    fname = min(fwd_alone, key=fwd_alone.get)
    aname = min(adj_alone, key=adj_alone.get)
    fb, fg, fo, fw = shapes[fname]
    ab, ag, _, aw = shapes[aname]
    ms_split = round(grad_ms(fb, fg, 1, fo, fw, adj=(ab, ag, aw)), 4)
    split_name = f"forward: {fname}; adjoint: {aname}"
    by_shape[split_name] = ms_split
    shapes[split_name] = (fb, fg, fo, fw)
    gshape = min(by_shape, key=by_shape.get)
    gb, gg, go, gw = shapes[gshape]
    gadj = (ab, ag, aw) if gshape == split_name else (gb, gg, gw)
    per_k = {1: by_shape[gshape]}
    for k in (8, 32, 128):
        per_k[k] = round(grad_ms(gb, gg, k, go, adj=gadj), 4)
    best = min(per_k.items(), key=lambda kv: kv[1])
    # accuracy of the forward (final state) against Verner 7 at 1e-13, 10,000 orbits
    idx = np.sort(np.random.default_rng(19).choice(n, 10_000, replace=False))
    ws = subset(wg, idx)
    ref = api.solve(mk(api, ws, tableau="verner7", rtol=1e-13, atol=1e-13))
    torch.cuda.synchronize()
    eps = orbit_error(plain.y_final.cpu().numpy()[:, idx], ref.y_final.cpu().numpy(),
                      ws["y0"], ws["theta"])
    # the adjoint kernel alone (store-mode tape, HIP events on its stream)
    cap1 = nmax + 2
    fused = api.Solution(pg, api.Launch(block=gb, grid=gg, ckpt_every=1, ckpt_capacity=cap1,
                                        wide=gw))
    fused.set_order(gorder)
    fused.run()
    ybf[0, :3] = 2.0 * (fused.y_final[:3] - T)
    steps_g = int(fused.n_accepted.to(torch.int64).sum())
    ms_vjp = timed(lambda: api.solve_vjp(fused, ybar_final=ybf, block=gadj[0], grid=gadj[1],
                                         wide=gadj[2]), reps, 1, torch)
    fvs = FLOPS_PER_VJP_STEP[("dopri5", "loghalo")]
    ach_vjp = steps_g * fvs / (ms_vjp * 1e-3) / 1e12
    i_g = int(torch.argmax(fused.n_accepted))
    p1 = mk(api, subset(wg, [i_g]))
    s1 = api.Solution(p1, api.Launch(block=64, ckpt_every=1, ckpt_capacity=cap1))
    ms_f1 = timed(lambda: s1.run(), 3, 1, torch)
    yb1 = torch.ones((1, 6, 1), dtype=torch.float64, device="cuda")
    ms_v1 = timed(lambda: api.solve_vjp(s1, ybar_final=yb1), 3, 1, torch)
    ms_v1g = timed(lambda: api.solve_vjp(s1, ybar_final=yb1, wide=1), 3, 1, torch)
    vjp_roofline = {"kernel": "gs::vjp_kernel<Dopri5, LogHalo>, store-mode tape",
                    "launch": aname if gshape == split_name else gshape, "bound": "alu",
                    "flops_per_accepted_step": fvs,
                    "accepted_steps": steps_g, "ms": round(ms_vjp, 4),
                    "achieved": round(ach_vjp, 3), "peak": PEAK_FP64_VECTOR_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(ach_vjp / PEAK_FP64_VECTOR_TFLOPS, 4),
                    "critical_path": {
                        "max_accepted_one_orbit": int(fused.n_accepted.max()),
                        "longest_alone_ms": {"forward_with_tape": round(ms_f1, 3),
                                             "adjoint": round(ms_v1, 3),
                                             "adjoint_on_a_group": round(ms_v1g, 3)},
                        "batch_adjoint_over_longest_alone": round(ms_vjp / ms_v1, 3)}}
    log(f"[bench] c3: forward {ms_fwd:.3f} ms, gradient {best[1]:.3f} ms ({gshape}, k = "
        f"{best[0]}), adjoint alone {ms_vjp:.3f} ms ({ach_vjp / PEAK_FP64_VECTOR_TFLOPS:.1%}), "
        f"longest orbit's adjoint alone {ms_v1:.3f} ms ({ms_v1g:.3f} ms on a group); "
        f"alone by launch {adj_alone}")
    del fused, s1
    # forward sensitivities (the paper's own derivative), 2 and 9 columns, one
    # lane per orbit or the longest 256 on 16-lane groups (the batch is bound
    # by its longest orbit), reported at the faster
    sens = {}
    for cols in ([6, 7], list(range(9))):
        by = {}
        for lname, L in (("lanes", api.Launch()), ("256 on groups", api.Launch(wide=256))):
            by[lname] = round(timed(lambda: api.solve_sens(pg, cols, L, order=gorder), reps, 1,
                                    torch), 4)
        fast = min(by, key=by.get)
        sens[str(len(cols))] = {"ms": by[fast], "ratio": round(by[fast] / ms_fwd, 3),
                                "launch": fast, "ms_by_launch": by}
    log(f"[bench] c3 forward sensitivities: 2 columns {sens['2']['ms']:.3f} ms "
        f"({sens['2']['ratio']:.2f}x the forward, {sens['2']['launch']}; "
        f"{sens['2']['ms_by_launch']}), 9 columns {sens['9']['ms']:.3f} ms "
        f"({sens['9']['ratio']:.2f}x)")
    res = {"workload": "100,000 orbits to t = 100, Dopri5 1e-8 / 1e-10, loss sum |x - T|^2, "
                       "gradient with respect to (v0, q, rc) and the initial conditions",
           "ms_forward": round(ms_fwd, 4), "ms_gradient": round(best[1], 4),
           "grad_forward_ratio": best[1] / ms_fwd, "gradient_launch": gshape,
           "ckpt_every": best[0], "ms_gradient_by_launch": by_shape, "ms_by_ckpt_every": per_k,
           "ms_alone_by_launch": {"forward_with_tape": fwd_alone, "adjoint": adj_alone},
           "accuracy": accuracy_row(eps, ORBIT_BUDGET, "eq:st-fwderr, final state",
                                    "Verner 7 at 1e-13 on the GPU, 10,000 orbits"),
           "vjp_roofline": vjp_roofline, "forward_sensitivities_by_columns": sens}
    return res


def gradient_profile(args, torch, api, inputs):
    """`--mode gradient`: the gradient workload's fastest launch (store-mode
    tape, device order, 256-lane workgroups, one wave per SIMD), forward with
    tape then adjoint, `--steps` times after `--warmup`, for kernel traces."""
    wg = inputs.orbits_gradient()
    pg = mk(api, wg)
    T = torch.as_tensor(wg["targets"], device="cuda")
    plain = api.Solution(pg, api.Launch())
    order = plain.queue_order().clone()
    plain.set_order(order)
    plain.run()
    torch.cuda.synchronize()
    nmax = int(plain.n_accepted.max())
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    taped = api.Solution(pg, api.Launch(block=256, grid=cus, ckpt_every=1,
                                        ckpt_capacity=nmax + 2))
    taped.set_order(order)
    ybf = torch.zeros((1, 6, pg.n), dtype=torch.float64, device="cuda")

    def step():
        taped.run()
        ybf[0, :3] = 2.0 * (taped.y_final[:3] - T)
        api.solve_vjp(taped, ybar_final=ybf, block=256, grid=cus)

    ms = timed(step, args.steps, args.warmup, torch)
    print(json.dumps({"mode": "gradient", "ms_per_step": ms, "steps": args.steps}))


# ---- c5: cosmologies ----------------------------------------------------------------------

def c5_quint(args, torch, api, inputs):
    res = {}
    for dense in (False, True):
        w = inputs.quintessence(dense=dense)
        prob = mk(api, w)
        sol = api.Solution(prob, api.Launch())
        graph = api.Graph(sol)
        ms = timed(lambda: graph.launch(), 20, 3, torch)
        ref = api.solve(mk(api, w, tableau="verner7", rtol=1e-11, atol=1e-13))
        torch.cuda.synchronize()
        a0, lam, om, orad = w["theta"]
        N = w["t_out"][:, None]

        def dist(yo, yf):
            E = np.sqrt((om * np.exp(-3 * N) + orad * np.exp(-4 * N)
                         + a0 * np.exp(-lam * yo[0])) / (1 - yo[1] ** 2 / 6))
            return yf[2][None, :] - yo[2], 1.0 / E

        dm, dh = dist(sol.y_out.cpu().numpy(), sol.y_final.cpu().numpy())
        rm, rh = dist(ref.y_out.cpu().numpy(), ref.y_final.cpu().numpy())
        eps = np.maximum(np.abs(dm - rm), np.abs(dh - rh)).max(axis=0)
        key = "nodes_64" if dense else "nodes_7"
        res[key] = {"ms": round(ms, 4), "solves_per_s": prob.n / (ms * 1e-3),
                    "accuracy": accuracy_row(eps, DE_BUDGET, "max |dD_M|, |dD_H| (c/H0)",
                                             "Verner 7 at 1e-11 / 1e-13 on the GPU")}
        graph.close()
        log(f"[bench] c5 {key}: {ms:.4f} ms, P99 {p99(eps):.2e}")
    res["workload"] = ("10,000 cosmologies, lambda ~ U[0, 1.5], Omega_m ~ U[0.28, 0.34], "
                       "Dopri5 1.78e-4 / 1.78e-7, distances at 7 (or 64) redshifts")
    res["profile"] = de_profile(args, torch, api, inputs)
    return res


def de_profile(args, torch, api, inputs):
    wd = inputs.de_profile_mocks()
    f = wd["fid"]
    kw = dict(newton=wd["newton"], mu=wd["mu"], trust=wd["trust"], rtol=wd["rtol"],
              atol=wd["atol"], N_start=wd["t0"])
    kw["N_data"] = wd["N_nodes"]
    K = len(wd["N_nodes"])
    fid = api.de_profile([f["lam"]], [f["om"]], [f["h"]], [1.0 - f["om"] - wd["omega_r"]],
                         wd["omega_r"], wd["N_spline"], np.zeros((2, K, 1)), np.ones((2, K)),
                         iters=0, **kw)
    dfid = fid["dist"][:, :, 0]
    nm, nl = wd["eps"].shape[0], len(wd["lam_grid"])
    nfit = nm * nl
    eps = torch.as_tensor(wd["eps"], device="cuda")[torch.arange(nfit, device="cuda") // nl]
    data = (dfid[:, :, None] * (1.0 + wd["rel_noise"] * eps.permute(1, 2, 0))).contiguous()
    sigma = (wd["rel_noise"] * dfid).contiguous()
    dev = dict(dtype=torch.float64, device="cuda")
    lam = torch.as_tensor(np.tile(wd["lam_grid"], nm), **dev)
    om0 = torch.full((nfit,), wd["start"]["om"], **dev)
    h0 = torch.full((nfit,), wd["start"]["h"], **dev)
    a00 = 1.0 - om0 - wd["omega_r"]
    Nn = torch.as_tensor(wd["N_spline"], **dev)
    prof = {"workload": f"{nm} mocks x {nl} slopes = {nfit} Gauss-Newton fits, "
                        f"{wd['iters']} iterations, 64 solver nodes, spline to 7 data redshifts"}
    a0_flat = api.de_profile(lam, om0, h0, a00, wd["omega_r"], Nn, data, sigma, iters=0,
                             **kw)["a0"]
    for name, newton, a0s in (("a0_solved", wd["newton"], a00), ("a0_supplied", 0, a0_flat)):
        def profile():
            return api.de_profile(lam, om0, h0, a0s, wd["omega_r"], Nn, data, sigma,
                                  iters=wd["iters"], **dict(kw, newton=newton))

        ms_p = timed(profile, 5, 1, torch)
        res = profile()
        torch.cuda.synchronize()
        conv = ((res["chi2_prev"] - res["chi2"]).abs() < 1e-4) & (res["decrement"].abs() < 1e-6)
        us_it = ms_p * 1e3 / (nfit * wd["iters"])
        prof[name] = {"newton_steps": newton, "ms": round(ms_p, 4),
                      "us_per_iteration_per_fit": round(us_it, 4),
                      "converged_fraction": round(float(conv.float().mean()), 4),
                      "all_ok": bool((res["status"] == 0).all())}
        log(f"[bench] dark-energy profile ({name}): {ms_p:.3f} ms")
    return prof


# ---- the stiff path ----------------------------------------------------------------------

def rodas4_flops_per_attempt(D, jac_flops, rhs_flops):
    """Algorithmic FP64 flops of one Rodas4 attempt of the stiff kernel (fma =
    2, division or reciprocal = 1): Jacobian; the matrix 1/(h gamma) I - J
    (D + 2); LU with partial pivoting, sum over columns of m multipliers and
    m^2 updates, m = D-1..0, plus D pivot reciprocals; six triangular solves
    of 2 D^2 - D each; stage sums 70 D + 1; six right-hand sides (five stages
    and f at the new point); y+ and the error norm 17 D + 1."""
    lu = sum(m + 2 * m * m for m in range(D)) + D
    return (jac_flops + D + 2 + lu + 6 * (2 * D * D - D) + 70 * D + 1 + 6 * rhs_flops
            + 17 * D + 1)


# (generator, Jacobian flops, right-hand-side flops) of each stiff problem: the
# operations of the hand-written Jacobian and right-hand side as written.
STIFF = (("kinetics3", 3, 7), ("kinetics8", 6, 28), ("robertson", 5, 9), ("hires", 10, 41))


def stiff_features(torch, w, prob):
    """Features of the pilot cost model of a stiff ensemble, on the device: the
    logarithms of the rates, of the span (if it varies) and of every initial
    value that varies and stays positive."""
    rows = [torch.log(r) for r in prob.theta]
    if prob.t1.numel() > 1:
        rows.append(torch.log(prob.t1))
    for c in range(w["y0"].shape[0]):
        r = w["y0"][c]
        if np.all(r > 0) and np.ptp(r) > 0:
            rows.append(torch.log(prob.y0[c]))
    return torch.stack(rows)


def stiff_bench(torch, api, inputs, autotune):
    res = {}
    for gname, jac_f, rhs_f in STIFF:
        gen = getattr(inputs, gname)
        w = gen()
        prob = mk(api, w)
        feats = stiff_features(torch, w, prob)
        t_pilot, cost = wall_ms(lambda: autotune.pilot_cost(prob, feats), torch)
        tmp = api.Solution(prob, api.Launch())
        order = tmp.queue_order(cost).clone()
        del tmp
        sol = api.Solution(prob, autotune.tune_forward(prob, order=order, use_cache=False))
        sol.queue_order(cost)

        def body(stream):
            sol.queue_order(cost, stream=stream)
            sol.run(stream=stream)

        graph = api.Captured(body)
        ms = timed(graph.launch, 10, 2, torch)
        n = prob.n
        attempts = int((sol.n_accepted.to(torch.int64) + sol.n_rejected).sum())
        fpa = rodas4_flops_per_attempt(prob.d, jac_f, rhs_f)
        tf = fpa * attempts / (ms * 1e-3) / 1e12
        # accuracy: the same problem at rtol 1e-10, atol 1e-15 as reference, in units
        # of the solve's own error weights atol + rtol |y|
        ref = api.solve(mk(api, w, rtol=1e-10, atol=1e-15))
        torch.cuda.synchronize()
        yo, ro = sol.y_out.cpu().numpy(), ref.y_out.cpu().numpy()
        eps = (np.abs(yo - ro) / (w["atol"] + w["rtol"] * np.abs(ro))).max(axis=(0, 1))
        res[w["rhs"]] = {
            "workload": f"{n} {w['rhs']} trajectories, Rodas4 rtol {w['rtol']:g} atol "
                        f"{w['atol']:g}, 16 outputs, device order from a pilot-fitted cost",
            "ms": round(ms, 4), "solves_per_s": n / (ms * 1e-3), "attempts": attempts,
            "ms_order_setup": round(t_pilot, 2),
            "accuracy": accuracy_row(eps, 1.0, "max over components and outputs of |y - "
                                     "y_ref| / (atol + rtol |y_ref|) (tolerance units)",
                                     "Rodas4 at rtol 1e-10, atol 1e-15 on the GPU"),
            "roofline": {"bound": "alu", "flops_per_attempt": fpa, "achieved": round(tf, 3),
                         "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tf / PEAK_FP64_VECTOR_TFLOPS, 4)},
            "all_ok": bool((sol.status == 0).all())}
        log(f"[bench] stiff {w['rhs']}: {ms:.3f} ms, {tf / PEAK_FP64_VECTOR_TFLOPS:.1%} of peak, "
            f"P99 {p99(eps):.2f} tolerance units")
        del sol, graph, ref
        w = gen(n=1_000_000, K=0)
        prob = mk(api, w)
        feats = stiff_features(torch, w, prob)
        _, cost = wall_ms(lambda: autotune.pilot_cost(prob, feats), torch)
        tmp = api.Solution(prob, api.Launch())
        order = tmp.queue_order(cost).clone()
        del tmp
        sol = api.Solution(prob, autotune.tune_forward(prob, order=order, use_cache=False))
        ms = timed(lambda: (sol.queue_order(cost), sol.run()), 3, 1, torch)
        attempts = int((sol.n_accepted.to(torch.int64) + sol.n_rejected).sum())
        tf = fpa * attempts / (ms * 1e-3) / 1e12
        res[w["rhs"]]["at_1m"] = {"ms": round(ms, 4), "achieved": round(tf, 3),
                                  "frac": round(tf / PEAK_FP64_VECTOR_TFLOPS, 4),
                                  "all_ok": bool((sol.status == 0).all())}
        log(f"[bench] stiff {w['rhs']} at 10^6: {ms:.3f} ms ({tf / PEAK_FP64_VECTOR_TFLOPS:.1%})")
        del sol
    return res


# ---- precession gradients (configuration 4's 20,000-binary subset) ----------------------------

def precession_gradient(torch, api, inputs):
    w = inputs.spin_precession(n=20_000)
    n = w["y0"].shape[1]
    prob = mk(api, w, t_out=None)
    # 2x10^4 binaries fill under a third of the chip at one lane each, so the
    # head of the longest-first order (or every binary) may run on 16-lane
    # groups; each pass is reported at its faster launch
    tmp = api.Solution(prob, api.Launch())
    order = tmp.queue_order().clone()
    del tmp
    fwd_by = {}
    for name, L, o in (("lanes", api.Launch(), None),
                       ("half on groups", api.Launch(wide=n // 2), order)):
        s1 = api.Solution(prob, L)
        s1.set_order(o)
        fwd_by[name] = round(timed(lambda: s1.run(), 2, 1, torch), 2)
        del s1
    ms_f = min(fwd_by.values())
    plain = api.Solution(prob, api.Launch())
    plain.run()
    torch.cuda.synchronize()
    nmax = int(plain.n_accepted.max())
    # the forward with its tape on the faster forward launch; the adjoint on
    # single lanes (groups reverse more slowly)
    tape_wide = n // 2 if fwd_by["half on groups"] < fwd_by["lanes"] else 0
    sol = api.Solution(prob, api.Launch(ckpt_every=1, ckpt_capacity=nmax + 2, wide=tape_wide))
    sol.set_order(order if tape_wide else None)
    sol.run()
    y = sol.y_final.detach().clone().requires_grad_(True)
    ybar = torch.zeros((2, 9, n), dtype=torch.float64, device="cuda")
    for r, s0 in enumerate((3, 6)):
        a, b = y[0:3], y[s0:s0 + 3]
        ang = torch.atan2(torch.linalg.norm(torch.cross(a, b, dim=0), dim=0), (a * b).sum(0))
        (ybar[r],) = torch.autograd.grad(ang.sum(), y)

    def tilt_grads():
        sol.run()
        return api.solve_vjp(sol, ybar_final=ybar)

    ms_st = timed(tilt_grads, 1, 1, torch)
    tape_gb = sol.workspace.numel() / 1e9
    del sol
    sens_by = {}
    for name, L, o in (("lanes", api.Launch(), None),
                       ("all on groups", api.Launch(wide=n), order)):
        sens_by[name] = round(timed(lambda: api.solve_sens(prob, [9, 10, 11], L, order=o), 1, 1,
                                    torch), 2)
    ms_s = min(sens_by.values())
    res = {"workload": f"{n} binaries, r = 1000 -> 10, Verner 7 3.16e-9, losses: both final "
                       "tilt angles, parameters (q, chi1, chi2)",
           "ms_forward": round(ms_f, 2), "ms_forward_by_launch": fwd_by,
           "ms_forward_sensitivities_by_launch": sens_by,
           "ms_store_tape_plus_two_adjoints": round(ms_st, 2), "store_tape_gb": round(tape_gb, 1),
           "ratio_adjoint_store": round(ms_st / ms_f, 3),
           "ms_forward_sensitivities_3_columns": round(ms_s, 2),
           "ratio_forward_sensitivities": round(ms_s / ms_f, 3)}
    log(f"[bench] precession gradient: {json.dumps(res)}")
    del plain
    return res


# ---- the CPU oracle on the host -------------------------------------------------------------

def cpu_info():
    model, mhz = "unknown", None
    try:
        txt = open("/proc/cpuinfo").read()
        m = re.search(r"model name\s*:\s*(.+)", txt)
        model = m.group(1).strip() if m else model
        f = re.findall(r"cpu MHz\s*:\s*([0-9.]+)", txt)
        mhz = round(float(np.mean([float(x) for x in f])), 1) if f else None
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model, "mean_cpu_mhz": mhz}


def cpu_baseline(w, target_s=12.0):
    """The oracle as it is, on this host's cores (at most 16: the box's share),
    on a bounded seeded sample of the headline workload (all 32 outputs), and
    on one core."""
    import oracle

    threads = min(os.cpu_count() or 1, 16)
    n = w["y0"].shape[1]
    rng = np.random.default_rng(1234)

    def run(m, nt):
        idx = np.sort(rng.choice(n, m, replace=False))
        ws = subset(w, idx)
        t = time.perf_counter()
        o = oracle.solve(ws["rhs"], ws["tableau"], ws["y0"], ws["theta"], ws["t0"], ws["t1"],
                         ws["rtol"], ws["atol"], ws["t_out"], nthreads=nt)
        return time.perf_counter() - t, o

    dt1, o1 = run(8, 1)
    m1 = int(max(8, min(200, 8 * (target_s / 2) / max(dt1, 1e-3))))
    dt1, o1 = run(m1, 1)
    m = int(max(threads, min(20_000, m1 * threads * target_s / max(dt1, 1e-3))))
    dt, o = run(m, threads)
    info = cpu_info()
    att = int((o["n_accepted"] + o["n_rejected"]).sum())
    return {"value": m / dt, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"{m} seeded binaries of the headline workload (r = 1000 -> 10, Verner 7 "
                      f"at 1e-11, 32 outputs; {att} attempts), {dt:.1f} s wall on {threads} "
                      "threads",
            "one_core": {"value": m1 / dt1, "unit": "solves/s", "sample": f"{m1} binaries, "
                         f"{dt1:.1f} s"},
            "us_per_binary": {"all_cores": round(dt / m * 1e6, 1),
                              "one_core": round(dt1 / m1 * 1e6, 1)},
            "host": info}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures exactly one GPU; --gpus {args.gpus} is not supported "
              "(trajectories are independent; a multi-GPU run would split them by index).",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2609_28458_amd import api, autotune, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    api.lib()
    dev_name = torch.cuda.get_device_name(0)

    if args.mode == "gradient":
        gradient_profile(args, torch, api, inputs)
        return
    if args.mode == "traffic":
        # A device copy of exactly 1 GiB calibrates FETCH_SIZE / WRITE_SIZE.
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        del a, b
    w, prob, sol, graph, cost, pilot_ms = headline(args, torch, api, inputs, autotune)
    if args.mode == "traffic":
        graph.launch()
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": (1 << 27) * 8, "kernel_source_sha": kernel_source_sha()}))
        return
    if args.mode == "profile":
        ms = timed(graph.launch, args.steps, args.warmup, torch)
        print(json.dumps({"mode": "profile", "ms_per_step": ms, "steps": args.steps}))
        return
    if args.mode == "lone":
        graph.launch()
        torch.cuda.synchronize()
        i_long = int(torch.argmax(sol.n_accepted + sol.n_rejected))
        lsol = api.Solution(mk(api, subset(w, [i_long])), api.Launch(block=64))
        lsol.run()
        torch.cuda.synchronize()
        print(json.dumps({"attempts": int((lsol.n_accepted + lsol.n_rejected).item())}))
        return

    out, ms = headline_rows(args, torch, api, inputs, autotune, w, prob, sol, graph, cost,
                            pilot_ms)
    out["device"] = dev_name
    del sol, graph
    torch.cuda.empty_cache()
    if not args.no_rest:
        out["c2_uneven_orbits"] = c2_uneven(args, torch, api, inputs, autotune)
        torch.cuda.empty_cache()
        out["c1_orbits"] = c1_forward(torch, api, inputs, autotune)
        torch.cuda.empty_cache()
        c3 = c3_gradient(torch, api, inputs, autotune)
        out["c3_gradient"] = c3
        out["grad_forward_ratio"] = c3["grad_forward_ratio"]
        torch.cuda.empty_cache()
        out["c5_cosmologies"] = c5_quint(args, torch, api, inputs)
        torch.cuda.empty_cache()
        out["stiff"] = stiff_bench(torch, api, inputs, autotune)
        torch.cuda.empty_cache()
        out["c4_gradient_subset"] = precession_gradient(torch, api, inputs)
        torch.cuda.empty_cache()
    if not args.no_cpu:
        cb = cpu_baseline(w)
        out["cpu_baseline"] = cb
        log(f"[bench] cpu oracle: {cb['value']:.1f} solves/s on {cb['cores']} threads, "
            f"{cb['one_core']['value']:.2f} on one core ({cb['host']['model']})")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
