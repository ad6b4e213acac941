"""Benchmark: ensemble solve throughput on one MI355X.

Headline workload (N = 1): the uneven batch of 100,000 orbits in the
flattened logarithmic halo with per-orbit (v0, q, rc), t_end ~ logU[10, 500]
and rtol ~ logU[1e-9, 1e-6] (atol = rtol), Tsit5, final states.  One step is
one complete ensemble solve from device-resident inputs: the work-queue
reset and the persistent solve kernel, captured once in a hipGraph and
replayed; the launch shape comes from the autotuner.  `value` is solves per
second.

Also reported on the same line:
  * accepted RK steps/s and step attempts/s of the headline run;
  * roofline of the solve kernel: algorithmic FP64 flops per launch over its
    duration (HIP events on the launch stream) against the FP64 vector peak,
    HBM traffic from the committed PMC summary when it matches the kernel
    source, and the critical path of this batch (its longest orbit solved
    alone, on one lane and on one 16-lane group, the faster of the two,
    against the batch's time);
  * the same kernel at full occupancy (10^6 uniform orbits) for comparison;
  * the two other launch arms of the batch (static one lane per trajectory,
    one launch per cost bucket);
  * the grad/forward time ratio on the gradient workload (100,000 orbits to
    t = 100, Dopri5 1e-8/1e-10, loss sum |x - T|^2): forward with tape plus
    adjoint, over the forward without tape;
  * cpu_baseline: the CPU oracle on a bounded sample of the same batch.

Modes: `--mode profile` runs the headline steps only (for rocprofv3 kernel
traces); `--mode traffic` runs one device copy of known size and one headline
solve (for rocprofv3 FETCH_SIZE / WRITE_SIZE passes); `--mode lone` runs the
batch's longest orbit alone on one lane and on one 16-lane group (for
per-dispatch instruction counters).
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
#   Verner 7 + precession (d 9, s 10, nnz(A) 36, nnz(b) 7, nnz(e) 8, 119 per evaluation):
#   810 + 144 + 18 + 153 + 47 + 5 + 1190 = 2367; one output node (a shortened step) adds
#   9 evaluations and the stage sums and update, 1071 + 810 + 144 = 2025.
FLOPS_PER_ATTEMPT = {("tsit5", "loghalo"): 541, ("dopri5", "loghalo"): 517,
                     ("verner7", "spinprec"): 2367}
FLOPS_PER_NODE = {("verner7", "spinprec"): 2025, ("dopri5", "loghalo"): 168}
# Reverse of one accepted step (store-mode tape, one loss): recompute the first
# right-hand side, the stage points and right-hand sides of the stages that feed
# the step, then seed h b_j lam, reverse every feeding stage through the
# right-hand side's VJP (46 flops for the log halo) and the transposed stage sums.
FLOPS_PER_VJP_STEP = {("dopri5", "loghalo"): 880}
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles",
                               "traffic_solve_kernel_tsit5_loghalo_orbits_uneven_100k.md")
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--mode", choices=("full", "profile", "traffic", "lone"), default="full")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-grad", action="store_true", help="skip the gradient ratio")
    ap.add_argument("--no-arms", action="store_true", help="skip the static and bucket arms")
    return ap.parse_args()


def timed(fn, steps, warmup, torch):
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
    return start.elapsed_time(stop) / steps  # ms per step


def cpu_baseline(w, target_thread_seconds=15.0):
    """The oracle as it is, on this host's cores, on a bounded seeded sample."""
    import oracle

    threads = min(os.cpu_count() or 1, 16)
    rng = np.random.default_rng(1234)
    n = w["y0"].shape[1]

    def run(m):
        idx = np.sort(rng.choice(n, m, replace=False))
        t = time.perf_counter()
        o = oracle.solve(w["rhs"], w["tableau"], w["y0"][:, idx], w["theta"][:, idx], 0.0,
                         w["t1"][idx], w["rtol"][idx], w["atol"][idx], nthreads=threads)
        return time.perf_counter() - t, o

    m = 2000
    dt, _ = run(m)
    m = int(min(n, max(m, m * target_thread_seconds / threads / max(dt, 1e-3))))
    dt, o = run(m)
    res = {"value": m / dt, "unit": "solves/s", "cores": threads, "kind": "oracle",
           "sample": f"{m} seeded orbits of the 100,000-orbit uneven batch "
                     f"({int(o['n_accepted'].sum())} accepted steps), {dt:.2f} s wall on "
                     f"{threads} threads"}
    # the stiff path's oracle on 5,000 seeded trajectories of each kinetics workload
    from paper_2609_28458_amd import inputs
    stiff = {}
    for gen in (inputs.kinetics3, inputs.kinetics8):
        ws = gen()
        idx = np.sort(np.random.default_rng(77).choice(ws["y0"].shape[1], 5000, replace=False))
        t0 = time.perf_counter()
        oracle.solve(ws["rhs"], "rodas4", ws["y0"][:, idx], ws["theta"][:, idx], 0.0,
                     ws["t1"][idx], ws["rtol"], ws["atol"], ws["t_out"][:, idx],
                     nthreads=threads)
        stiff[ws["rhs"]] = round(5000 / (time.perf_counter() - t0), 1)
    res["stiff_oracle_solves_per_s"] = stiff
    return res


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


def stiff_bench(args, torch, api, inputs, autotune):
    """Rodas4 kernel on the two stiff kinetics workloads (10^5 trajectories,
    16 output times each), graph-launched; at 10^6 trajectories for the
    throughput."""
    res = {}
    for gen, jac_f, rhs_f in ((inputs.kinetics3, 3, 7), (inputs.kinetics8, 6, 28)):
        w = gen()
        prob = api.make_problem(w["rhs"], w["tableau"], w["y0"], w["theta"], w["t0"], w["t1"],
                                w["rtol"], w["atol"], w["t_out"])
        # longest first by a cost model fitted on a pilot solve of 4,096 trajectories
        # (step attempts against the logs of the rates, span and varying initial values)
        feats = ([np.log(r) for r in w["theta"]] + [np.log(w["t1"])]
                 + [np.log(r) for r in w["y0"] if np.all(r > 0) and np.ptp(r) > 0])
        sorder = autotune.pilot_order(prob, feats)
        sol = api.Solution(prob, autotune.tune_forward(prob, order=sorder, use_cache=False))
        sol.set_order(sorder)
        graph = api.Graph(sol)
        ms = timed(lambda: graph.launch(), max(5, args.steps // 2), 2, torch)
        torch.cuda.synchronize()
        n = prob.n
        attempts = int((sol.n_accepted.to(torch.int64) + sol.n_rejected).sum())
        ok = bool((sol.status == 0).all())
        fpa = rodas4_flops_per_attempt(prob.d, jac_f, rhs_f)
        tf = fpa * attempts / (ms * 1e-3) / 1e12
        res[w["rhs"]] = {
            "workload": f"{n} stiff {w['rhs']} trajectories, Rodas4 rtol {w['rtol']:g} atol "
                        f"{w['atol']:g}, 16 outputs, longest first by a pilot-fitted cost "
                        "model", "ms": round(ms, 4),
            "solves_per_s": n / (ms * 1e-3), "attempts": attempts, "all_ok": ok,
            "roofline": {"bound": "alu", "flops_per_attempt": fpa, "achieved": round(tf, 3),
                         "peak": 78.6, "unit": "TFLOP/s", "frac": round(tf / 78.6, 4)},
            "launch": {k: sol.launch.__dict__[k] for k in ("block", "grid", "refill")}}
        log(f"[bench] stiff {w['rhs']}: {ms:.3f} ms, {n / ms * 1e3:.3e} solves/s, "
            f"{tf:.2f} TFLOP/s ({tf / 78.6:.1%} of FP64 peak)")
        graph.close()
        del sol, graph
        # ten times the trajectories: enough lanes to fill every SIMD several times over,
        # in the same kind of order
        w = gen(n=1_000_000, K=0)
        prob = api.make_problem(w["rhs"], w["tableau"], w["y0"], w["theta"], w["t0"], w["t1"],
                                w["rtol"], w["atol"])
        feats = ([np.log(r) for r in w["theta"]] + [np.log(w["t1"])]
                 + [np.log(r) for r in w["y0"] if np.all(r > 0) and np.ptp(r) > 0])
        sorder = autotune.pilot_order(prob, feats)
        sol = api.Solution(prob, autotune.tune_forward(prob, order=sorder, use_cache=False))
        sol.set_order(sorder)
        ms = timed(lambda: sol.run(), 3, 1, torch)
        attempts = int((sol.n_accepted.to(torch.int64) + sol.n_rejected).sum())
        tf = fpa * attempts / (ms * 1e-3) / 1e12
        res[w["rhs"]]["full_chip"] = {"workload": "1,000,000 trajectories, final state only, "
                                                  "longest first by a pilot-fitted cost model",
                                      "ms": round(ms, 4), "achieved": round(tf, 3),
                                      "frac": round(tf / 78.6, 4)}
        log(f"[bench] stiff {w['rhs']} at 10^6: {ms:.3f} ms, {tf:.2f} TFLOP/s "
            f"({tf / 78.6:.1%})")
        del sol
    return res


def precession_showcase(torch, api, inputs, autotune):
    """10^6 binaries from r = 1000 to 10, Verner 7 at 3.16e-9, 32 outputs: the
    configuration whose work keeps every SIMD busy for seconds, timed once
    after one warm-up run.  Binaries take 12,000 to 88,000 attempts, so they
    run longest first by a cost model fitted on a pilot solve of 4,096 of
    them (features: log q, both spin magnitudes, and the cosines between the
    orbital and spin directions)."""
    w = inputs.spin_precession(n=1_000_000)
    n = w["y0"].shape[1]
    prob = api.make_problem(w["rhs"], w["tableau"], w["y0"], w["theta"], w["t0"], w["t1"],
                            w["rtol"], w["atol"], w["t_out"])
    y, th = w["y0"], w["theta"]
    feats = [np.log(th[0]), th[1], th[2], (y[0:3] * y[3:6]).sum(0), (y[0:3] * y[6:9]).sum(0),
             (y[3:6] * y[6:9]).sum(0)]
    order = autotune.pilot_order(prob, feats)
    sol = api.Solution(prob, api.Launch())
    sol.set_order(order)
    ms = timed(lambda: sol.run(), 1, 1, torch)
    attempts = int((sol.n_accepted.to(torch.int64) + sol.n_rejected).sum())
    flops = (attempts * FLOPS_PER_ATTEMPT[("verner7", "spinprec")]
             + n * prob.K * FLOPS_PER_NODE[("verner7", "spinprec")])
    tf = flops / (ms * 1e-3) / 1e12
    res = {"workload": f"{n} binaries, r = 1000 -> 10, Verner 7 3.16e-9, {prob.K} outputs, "
                       "longest first by a pilot-fitted cost model",
           "ms": round(ms, 2), "attempts": attempts,
           "flops_per_attempt": FLOPS_PER_ATTEMPT[("verner7", "spinprec")],
           "achieved": round(tf, 3), "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
           "frac": round(tf / PEAK_FP64_VECTOR_TFLOPS, 4),
           "all_ok": bool((sol.status == 0).all())}
    log(f"[bench] precession showcase: {ms:.1f} ms, {attempts} attempts, {tf:.2f} TFLOP/s "
        f"({tf / PEAK_FP64_VECTOR_TFLOPS:.1%})")
    del sol
    return res


def precession_gradient(torch, api, inputs):
    """Gradients of both final tilt angles with respect to (q, chi1, chi2) for
    2x10^4 binaries from r = 1000: the forward solve alone, the forward with a
    checkpoint tape plus one adjoint launch per loss, and the paper's own
    route, forward sensitivities of the three parameters."""
    w = inputs.spin_precession(n=20_000)
    n = w["y0"].shape[1]
    prob = api.make_problem(w["rhs"], w["tableau"], w["y0"], w["theta"], w["t0"], w["t1"],
                            w["rtol"], w["atol"])
    plain = api.Solution(prob, api.Launch())
    ms_f = timed(lambda: plain.run(), 2, 1, torch)
    cap = int(plain.n_accepted.max()) // 128 + 2
    sol = api.Solution(prob, api.Launch(ckpt_every=128, ckpt_capacity=cap))
    # cotangents of the two tilt angles at the (deterministic) final state, once
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

    ms_g = timed(tilt_grads, 1, 1, torch)
    del sol
    # store mode: every accepted step on the tape (tens of GB here), no replay
    sol = api.Solution(prob, api.Launch(ckpt_every=1,
                                        ckpt_capacity=int(plain.n_accepted.max()) + 2))
    tape_gb = sol.workspace.numel() / 1e9
    ms_st = timed(tilt_grads, 1, 1, torch)
    ms_s = timed(lambda: api.solve_sens(prob, [9, 10, 11]), 1, 1, torch)
    res = {"workload": f"{n} binaries, r = 1000 -> 10, Verner 7 3.16e-9, losses: both final "
                       "tilt angles, parameters (q, chi1, chi2)",
           "ms_forward": round(ms_f, 2),
           "ms_tape_k128_plus_two_adjoints": round(ms_g, 2),
           "ratio_adjoint": round(ms_g / ms_f, 3),
           "ms_store_tape_plus_two_adjoints": round(ms_st, 2),
           "store_tape_gb": round(tape_gb, 1),
           "ratio_adjoint_store": round(ms_st / ms_f, 3),
           "ms_forward_sensitivities_3_columns": round(ms_s, 2),
           "ratio_forward_sensitivities": round(ms_s / ms_f, 3)}
    log(f"[bench] precession gradient: {json.dumps(res)}")
    del plain, sol
    return res


def paper_workloads(torch, api, inputs, autotune):
    """Microseconds per trajectory on the paper's three ensembles at 10^6
    trajectories, beside the figures the paper prints for one H200 NVL
    (context only: other hardware, and inputs drawn by this library's own
    recipes)."""
    res = {}
    # streams: forward, and forward with the sensitivities to (v_c, q) in the same launch
    w = inputs.streams()
    n = w["y0"].shape[1]
    prob = api.make_problem(w["rhs"], w["tableau"], w["y0"], w["theta"], w["t0"], w["t1"],
                            w["rtol"], w["atol"])
    sorder = np.argsort(-inputs.predicted_cost(w), kind="stable")
    launch = autotune.tune_forward(prob, order=sorder, use_cache=False)
    sol = api.Solution(prob, launch)
    sol.set_order(sorder)
    ms_f = timed(lambda: sol.run(), 5, 1, torch)
    att = (sol.n_accepted + sol.n_rejected).to(torch.float64).mean().item()
    ms_s = timed(lambda: api.solve_sens(prob, w["grad_cols"]), 3, 1, torch)
    res["streams"] = {"workload": f"{n} stream orbits, Tsit5 3.16e-7, 3.7 periods, final state "
                                  "(forward: longest first by dynamical times)",
                      "mean_attempts": round(att, 1),
                      "us_per_orbit_forward": round(ms_f * 1e3 / n, 5),
                      "us_per_orbit_with_sensitivities": round(ms_s * 1e3 / n, 5),
                      "paper_h200_us": {"forward": 0.12, "with_sensitivities": 0.22,
                                        "mean_attempts": 171}}
    del sol
    # dark-energy distances at 7 redshifts, amplitude supplied or solved for flatness
    w = inputs.quintessence(n=1_000_000)
    n = w["y0"].shape[1]
    prob = api.make_problem(w["rhs"], w["tableau"], w["y0"], w["theta"], w["t0"], w["t1"],
                            w["rtol"], w["atol"], w["t_out"])
    sol = api.Solution(prob, autotune.tune_forward(prob, use_cache=False))
    ms_a = timed(lambda: sol.run(), 5, 1, torch)
    del sol
    th = torch.as_tensor(w["theta"], device="cuda")
    K = len(w["t_out"])

    data = torch.zeros((2, K, n), dtype=torch.float64, device="cuda")
    sig = torch.ones((2, K), dtype=torch.float64, device="cuda")
    h1 = torch.ones_like(th[1])

    def solved():
        return api.de_profile(th[1], th[2], h1, th[0], float(w["theta"][3, 0]), w["t_out"], data,
                              sig, iters=0, newton=3, tableau=w["tableau"], N_start=w["t0"],
                              rtol=w["rtol"], atol=w["atol"])

    ms_b = timed(solved, 3, 1, torch)
    res["dark_energy"] = {"workload": f"{n} cosmologies, Dopri5 1.78e-4, 7 redshifts",
                          "us_per_cosmology_a0_supplied": round(ms_a * 1e3 / n, 5),
                          "us_per_cosmology_a0_solved": round(ms_b * 1e3 / n, 5),
                          "a0_solved_includes": "3 Newton solves with S_a0, then the distances "
                                                "with their derivative along flat models",
                          "paper_h200_us": {"a0_supplied": 0.0037, "a0_solved": 0.051}}
    # spin precession in the paper's setting, r = 100 -> 10
    w = inputs.spin_precession(n=1_000_000)
    n = w["y0"].shape[1]
    prob = api.make_problem(w["rhs"], w["tableau"], w["y0"], w["theta"], 100.0 ** -0.5, w["t1"],
                            w["rtol"], w["atol"])
    y, th = w["y0"], w["theta"]
    porder = autotune.pilot_order(prob, [np.log(th[0]), th[1], th[2], (y[0:3] * y[3:6]).sum(0),
                                         (y[0:3] * y[6:9]).sum(0), (y[3:6] * y[6:9]).sum(0)])
    sol = api.Solution(prob, api.Launch())
    sol.set_order(porder)
    ms_p = timed(lambda: sol.run(), 2, 1, torch)
    att = (sol.n_accepted + sol.n_rejected).to(torch.float64).mean().item()
    res["spin_precession"] = {"workload": f"{n} binaries, Verner 7 3.16e-9, r = 100 -> 10, "
                                          "longest first by a pilot-fitted cost model",
                              "mean_attempts": round(att, 1),
                              "us_per_binary": round(ms_p * 1e3 / n, 4),
                              "paper_h200_us": {"verner7": 3.2, "mean_attempts": 911}}
    del sol
    log(f"[bench] paper workloads: {json.dumps(res)}")
    return res


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


def headline(args, torch, api, inputs, autotune):
    w = inputs.orbits_uneven(n=args.n)
    prob = api.make_problem(w["rhs"], w["tableau"], w["y0"], w["theta"], w["t0"], w["t1"],
                            w["rtol"], w["atol"])
    order = np.argsort(-inputs.predicted_cost(w), kind="stable")
    return w, prob, order


def profile_launch(api):
    """A launch shape among the fastest the autotuner finds for the headline
    on MI355X (two wavefronts per workgroup, the occupancy-limited grid,
    refill at eight idle lanes, the 256 predicted-longest orbits on 16-lane
    groups), fixed for the profiling modes."""
    return api.Launch(schedule="queue", block=128, refill=8, wide=256)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures exactly one GPU; --gpus {args.gpus} is not supported "
              "(trajectories are independent; a multi-GPU run would split them by index).", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2609_28458_amd import api, autotune, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    api.lib()
    dev_name = torch.cuda.get_device_name(0)
    w, prob, order = headline(args, torch, api, inputs, autotune)
    n = prob.n

    if args.mode == "lone":
        # The batch's longest orbit alone, once on one lane and once on one 16-lane group
        # (for per-dispatch instruction counters: two dispatches of one wavefront each).
        sol = api.Solution(prob, profile_launch(api))
        sol.set_order(order)
        sol.run()
        i_long = int(torch.argmax(sol.n_accepted + sol.n_rejected))
        one = {k: (v[..., [i_long]] if isinstance(v, np.ndarray) and v.shape[-1:] == (n,)
                   else v) for k, v in w.items()}
        lprob = api.make_problem(one["rhs"], one["tableau"], one["y0"], one["theta"], one["t0"],
                                 one["t1"], one["rtol"], one["atol"])
        torch.cuda.synchronize()
        for wide in (0, 1):
            s1 = api.Solution(lprob, api.Launch(block=64, wide=wide))
            s1.run()
            torch.cuda.synchronize()
            print(json.dumps({"wide": wide, "attempts": int((s1.n_accepted + s1.n_rejected).item())}))
        return

    if args.mode == "traffic":
        # A device copy of exactly 1 GiB calibrates FETCH_SIZE / WRITE_SIZE.
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        sol = api.Solution(prob, profile_launch(api))
        sol.set_order(order)
        sol.run()
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 8, "kernel_source_sha": kernel_source_sha()}))
        return

    # ---- headline: autotuned persistent queue in a hipGraph, longest-first order -----------
    if args.mode == "full":
        launch = autotune.tune_forward(prob, order=order, use_cache=False)
    else:
        launch = profile_launch(api)
    sol = api.Solution(prob, launch)
    sol.set_order(order)
    graph = api.Graph(sol)
    ms = timed(lambda: graph.launch(), args.steps, args.warmup, torch)
    nacc = int(sol.n_accepted.to(torch.int64).sum())
    nrej = int(sol.n_rejected.to(torch.int64).sum())
    attempts = nacc + nrej
    max_att = int((sol.n_accepted + sol.n_rejected).max())
    ok = bool((sol.status == 0).all())
    log(f"[bench] {dev_name}: uneven batch n={n}: {ms:.3f} ms/solve, {attempts} attempts, "
        f"max per orbit {max_att}, all ok={ok}, launch {launch.__dict__}")
    if args.mode == "profile":
        graph.close()
        return

    # Kernel duration with HIP events on the launch stream (direct launches:
    # a one-thread counter reset and the solve kernel).
    s = torch.cuda.current_stream()

    def direct():
        sol.args.stream = s.cuda_stream
        api.gs_solve(sol.args)

    ms_kernel = timed(direct, args.steps, 1, torch)
    fpa = FLOPS_PER_ATTEMPT[("tsit5", "loghalo")]
    achieved = attempts * fpa / (ms_kernel * 1e-3) / 1e12

    # The critical path: the longest orbit of the batch alone, on one lane
    # and on one 16-lane group.  The batch cannot finish before that orbit
    # has run all of its attempts; alone on an idle chip it may run at a
    # lower clock than inside the loaded batch, so the ratio can dip below 1.
    i_long = int(torch.argmax(sol.n_accepted + sol.n_rejected))
    one = {k: (v[..., [i_long]] if isinstance(v, np.ndarray) and v.shape[-1:] == (n,) else v)
           for k, v in w.items()}
    lprob = api.make_problem(one["rhs"], one["tableau"], one["y0"], one["theta"], one["t0"],
                             one["t1"], one["rtol"], one["atol"])
    lsol = api.Solution(lprob, api.Launch(block=64))
    ms_lone = timed(lambda: lsol.run(), 3, 1, torch)
    us_per_attempt = ms_lone * 1e3 / max_att
    gsol = api.Solution(lprob, api.Launch(block=64, wide=1))
    ms_group = timed(lambda: gsol.run(), 3, 1, torch)
    us_group = ms_group * 1e3 / max_att
    assert int((gsol.n_accepted + gsol.n_rejected).item()) == max_att
    bound_ms = min(ms_lone, ms_group)

    traffic, traffic_src = committed_traffic()
    roofline = {"bound": "alu", "achieved": round(achieved, 3),
                "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_VECTOR_TFLOPS, 4), "traffic": traffic,
                "traffic_source": traffic_src,
                "kernel": "gs::solve_kernel<Tsit5, LogHalo, false, false>",
                "flops_per_attempt": fpa, "attempts_per_launch": attempts,
                "ms_per_launch": round(ms_kernel, 4),
                "critical_path": {"max_attempts_one_orbit": max_att,
                                  "longest_orbit_alone_ms": {"one_lane": round(ms_lone, 3),
                                                             "group": round(ms_group, 3)},
                                  "lone_wave_us_per_attempt": round(us_per_attempt, 4),
                                  "lone_group_us_per_attempt": round(us_group, 4),
                                  "longest_alone_ms": round(bound_ms, 3),
                                  "batch_over_longest_alone": round(ms_kernel / bound_ms, 3)}}

    # The same kernel with the chip full: 10^6 uniform orbits.
    nt = 1_000_000
    tw = inputs.orbits_uneven(n=nt, seed=6)
    tprob = api.make_problem(tw["rhs"], "tsit5", tw["y0"], tw["theta"], 0.0, np.full(nt, 20.0),
                             np.full(nt, 1e-8), np.full(nt, 1e-8))
    tw.update(t0=0.0, t1=np.full(nt, 20.0), rtol=np.full(nt, 1e-8), atol=np.full(nt, 1e-8))
    torder = np.argsort(-inputs.predicted_cost(tw), kind="stable")
    tsol = api.Solution(tprob, autotune.tune_forward(tprob, order=torder, use_cache=False))
    tsol.set_order(torder)
    ms_t = timed(lambda: tsol.run(), 3, 1, torch)
    att_t = int((tsol.n_accepted + tsol.n_rejected).to(torch.int64).sum())
    ach_t = att_t * fpa / (ms_t * 1e-3) / 1e12
    throughput = {"workload": "1,000,000 orbits, t = 20, rtol = atol = 1e-8, Tsit5, "
                              "longest-first by predicted dynamical times",
                  "launch": {k: tsol.launch.__dict__[k] for k in ("block", "grid", "refill",
                                                                   "wide")},
                  "ms": round(ms_t, 3), "attempts": att_t, "achieved": round(ach_t, 3),
                  "unit": "TFLOP/s", "frac": round(ach_t / PEAK_FP64_VECTOR_TFLOPS, 4)}
    # The 1,000-orbit forward recipe (shared halo, Dopri5 1e-8/1e-10, 64 outputs to t = 50)
    # at 10^6 orbits: its roofline with the chip full, outputs included.
    nc = 1_000_000
    cw = inputs.orbits_forward(n=nc, seed=1)
    cprob = api.make_problem(cw["rhs"], cw["tableau"], cw["y0"], cw["theta"], cw["t0"],
                             cw["t1"], cw["rtol"], cw["atol"], cw["t_out"])
    corder = np.argsort(-inputs.predicted_cost(cw), kind="stable")
    claunch = autotune.tune_forward(cprob, order=corder, use_cache=False)
    csol = api.Solution(cprob, claunch)
    csol.set_order(corder)
    ms_dkn = timed(lambda: csol.run(), 3, 1, torch)
    att_c = int((csol.n_accepted + csol.n_rejected).to(torch.int64).sum())
    del csol
    # the same with each trajectory's components of an output adjacent in y_out
    csol = api.Solution(cprob, api.Launch(**{**claunch.__dict__, "out_layout": "knd"}))
    csol.set_order(corder)
    ms_c = timed(lambda: csol.run(), 3, 1, torch)
    fl_c = (att_c * FLOPS_PER_ATTEMPT[("dopri5", "loghalo")]
            + nc * cprob.K * FLOPS_PER_NODE[("dopri5", "loghalo")])
    ach_c = fl_c / (ms_c * 1e-3) / 1e12
    c1_million = {"workload": "1,000,000 orbits of the 1,000-orbit forward recipe: shared halo, "
                              "Dopri5 1e-8/1e-10, 64 outputs to t = 50, longest-first",
                  "launch": {k: csol.launch.__dict__[k] for k in ("block", "grid", "refill")},
                  "out_layout": "[K][n][d]", "ms": round(ms_c, 3),
                  "ms_out_layout_dkn": round(ms_dkn, 3), "attempts": att_c,
                  "flops_per_attempt": FLOPS_PER_ATTEMPT[("dopri5", "loghalo")],
                  "flops_per_output": FLOPS_PER_NODE[("dopri5", "loghalo")],
                  "output_gb_per_s": round(6 * cprob.K * nc * 8 / (ms_c * 1e-3) / 1e9, 1),
                  "achieved": round(ach_c, 3), "unit": "TFLOP/s",
                  "frac": round(ach_c / PEAK_FP64_VECTOR_TFLOPS, 4),
                  "all_ok": bool((csol.status == 0).all())}
    log(f"[bench] 10^6 orbits, 64 outputs: {ms_c:.3f} ms, {ach_c:.2f} TFLOP/s "
        f"({100 * ach_c / PEAK_FP64_VECTOR_TFLOPS:.1f}%); [d][K][n] outputs {ms_dkn:.3f} ms")
    del csol
    torch.cuda.empty_cache()
    log(f"[bench] kernel {ms_kernel:.3f} ms = {achieved:.2f} TFLOP/s; lone wave "
        f"{us_per_attempt:.3f} us/attempt, lone group {us_group:.3f} us/attempt -> longest "
        f"orbit alone {bound_ms:.2f} ms; full chip "
        f"{ach_t:.2f} TFLOP/s")

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
        "config": {"workload": "orbits_uneven_100k", "n": n, "rhs": "loghalo",
                   "tableau": "tsit5", "rtol": "logU[1e-9,1e-6]", "t_end": "logU[10,500]",
                   "launch": "persistent queue, longest-first by predicted dynamical times, "
                             "head of the order on 16-lane groups, hipGraph, autotuned",
                   "block": launch.block, "grid": launch.grid, "refill": launch.refill,
                   "wide": launch.wide},
        "accepted_steps_per_s": nacc / (ms * 1e-3),
        "attempts_per_s": attempts / (ms * 1e-3),
        "all_trajectories_ok": ok,
        "device": dev_name,
        "roofline": roofline,
        "roofline_full_chip": throughput,
        "roofline_c1_million": c1_million,
    }

    # ---- the other two arms of the same batch -------------------------------------------
    if not args.no_arms:
        st = api.Solution(prob, api.Launch(schedule="static", block=256))
        ms_static = timed(lambda: st.run(), max(3, args.steps // 4), 1, torch)
        cost = inputs.predicted_cost(w)
        qs = np.quantile(cost, np.linspace(0, 1, 9))
        bucket_sols = []
        for b in range(8):
            sel = np.nonzero((cost >= qs[b]) & ((cost < qs[b + 1]) if b < 7 else True))[0]
            wb = {k: (v[..., sel] if isinstance(v, np.ndarray) and v.shape[-1] == n else v)
                  for k, v in w.items()}
            pb = api.make_problem(wb["rhs"], wb["tableau"], wb["y0"], wb["theta"], wb["t0"],
                                  wb["t1"], wb["rtol"], wb["atol"])
            bucket_sols.append(api.Solution(pb, api.Launch(schedule="static", block=256)))

        def buckets():
            for bs in bucket_sols:
                bs.run()

        ms_buckets = timed(buckets, max(3, args.steps // 4), 1, torch)
        out["arms_ms"] = {"persistent_graph": round(ms, 4), "static_one_lane_each":
                          round(ms_static, 4), "eight_cost_buckets": round(ms_buckets, 4)}
        log(f"[bench] arms: persistent {ms:.3f} ms, static {ms_static:.3f} ms, "
            f"buckets {ms_buckets:.3f} ms")

    # ---- gradient workload: grad/forward ratio --------------------------------------------
    if not args.no_grad:
        wg = inputs.orbits_gradient(n=args.n)
        pg = api.make_problem(wg["rhs"], wg["tableau"], wg["y0"], wg["theta"], wg["t0"],
                              wg["t1"], wg["rtol"], wg["atol"])
        reps = max(3, args.steps // 4)
        gorder = np.argsort(-inputs.predicted_cost(wg), kind="stable")
        T = torch.as_tensor(wg["targets"], device="cuda")
        # The forward alone at its best: the tuned launch (groups allowed), longest first.
        flaunch = autotune.tune_forward(pg, order=gorder, use_cache=False)
        plain = api.Solution(pg, flaunch)
        plain.set_order(gorder)
        ms_fwd = timed(lambda: plain.run(), reps, 1, torch)
        nmax = int(plain.n_accepted.max())
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        ybf = torch.zeros((1, 6, pg.n), dtype=torch.float64, device="cuda")

        def grad_ms(block, grid, k, order, wide=0):
            """Forward with tape, then the adjoint, in one launch shape."""
            taped = api.Solution(pg, api.Launch(block=block, grid=grid, ckpt_every=k,
                                                ckpt_capacity=nmax // k + 2, wide=wide))
            if order is not None:
                taped.set_order(order)

            def grad_step():
                taped.run()
                ybf[0, :3] = 2.0 * (taped.y_final[:3] - T)
                api.solve_vjp(taped, ybar_final=ybf, block=block, grid=grid)

            return timed(grad_step, reps, 1, torch)

        # The gradient at its best: store-mode tape in launch shapes with one or two waves
        # per SIMD (the persistent queues refill them), index or longest-first order, the
        # head of the order on 16-lane groups (which write the store-mode tape too); then
        # the checkpoint interval k in the best shape (single lanes only).
        shapes = {"block 256, occupancy grid, index order": (256, 0, None, 0),
                  "block 256, occupancy grid, longest first": (256, 0, gorder, 0),
                  "block 128, 2 waves per CU, longest first": (128, 2 * cus, gorder, 0),
                  "block 64, 1 wave per SIMD, longest first": (64, 4 * cus, gorder, 0),
                  "block 256, 1 wave per SIMD, longest first": (256, cus, gorder, 0),
                  "block 128, 2 waves per CU, longest first, 256 on groups":
                      (128, 2 * cus, gorder, 256),
                  "block 64, 1 wave per SIMD, longest first, 256 on groups":
                      (64, 4 * cus, gorder, 256)}
        by_shape = {name: round(grad_ms(sh[0], sh[1], 1, sh[2], sh[3]), 4)
                    for name, sh in shapes.items()}
        gshape = min(by_shape, key=by_shape.get)
        gb, gg, go, gw = shapes[gshape]
        per_k = {1: by_shape[gshape]}
        for k in (8, 32, 128):
            per_k[k] = round(grad_ms(gb, gg, k, go), 4)
        best = min(per_k.items(), key=lambda kv: kv[1])
        # the forward in the gradient's launch shape, for the ratio within one launch
        same = api.Solution(pg, api.Launch(block=gb, grid=gg, wide=gw))
        if go is not None:
            same.set_order(go)
        ms_fwd_same = timed(lambda: same.run(), reps, 1, torch)
        del same
        log(f"[bench] gradient: forward {ms_fwd:.3f} ms (tuned, longest first), gradient "
            f"{best[1]:.3f} ms ({gshape}, k = {best[0]}), by shape {by_shape}, by k {per_k}; "
            f"forward in that shape {ms_fwd_same:.3f} ms")
        # The plain arm: one lane per trajectory in both passes (static forward with the
        # store-mode tape; an adjoint grid with exactly one lane for every trajectory).
        cap1 = int(plain.n_accepted.max()) + 2
        fused = api.Solution(pg, api.Launch(block=256, ckpt_every=1, ckpt_capacity=cap1))
        stat = api.Solution(pg, api.Launch(schedule="static", block=256, ckpt_every=1,
                                           ckpt_capacity=cap1))
        ybf = torch.zeros((1, 6, pg.n), dtype=torch.float64, device="cuda")
        grads = {}

        def grad_of(sol, grid):
            def step():
                sol.run()
                ybf[0, :3] = 2.0 * (sol.y_final[:3] - T)
                grads[grid] = api.solve_vjp(sol, ybar_final=ybf, grid=grid)
            return step

        ms_stat = timed(grad_of(stat, (pg.n + 255) // 256), max(3, args.steps // 4), 1, torch)
        ms_fused = timed(grad_of(fused, 0), max(3, args.steps // 4), 1, torch)
        same = all(torch.equal(a, b) for a, b in zip(grads[0], grads[(pg.n + 255) // 256]))
        log(f"[bench] gradient arms: fused persistent {ms_fused:.3f} ms, one lane per trajectory "
            f"{ms_stat:.3f} ms, identical gradients {same}")
        # The adjoint kernel alone (store-mode tape, HIP events on its stream): algorithmic
        # flops are the per-accepted-step count of the reverse step times the accepted steps.
        fused.run()
        ybf[0, :3] = 2.0 * (fused.y_final[:3] - T)
        steps_g = int(fused.n_accepted.to(torch.int64).sum())
        ms_vjp = timed(lambda: api.solve_vjp(fused, ybar_final=ybf), max(3, args.steps // 4), 1,
                       torch)
        fvs = FLOPS_PER_VJP_STEP[("dopri5", "loghalo")]
        ach_vjp = steps_g * fvs / (ms_vjp * 1e-3) / 1e12
        vjp_roofline = {"kernel": "gs::vjp_kernel<Dopri5, LogHalo>, store-mode tape",
                        "bound": "alu", "flops_per_accepted_step": fvs,
                        "accepted_steps": steps_g, "ms": round(ms_vjp, 4),
                        "achieved": round(ach_vjp, 3), "peak": PEAK_FP64_VECTOR_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(ach_vjp / PEAK_FP64_VECTOR_TFLOPS, 4)}
        # Its critical path: the longest orbit of the workload alone (forward with tape,
        # then the adjoint).
        i_g = int(torch.argmax(fused.n_accepted))
        one_g = {k: (v[..., [i_g]] if isinstance(v, np.ndarray) and v.shape[-1:] == (pg.n,)
                     else v) for k, v in wg.items()}
        p1 = api.make_problem(one_g["rhs"], one_g["tableau"], one_g["y0"], one_g["theta"],
                              one_g["t0"], one_g["t1"], one_g["rtol"], one_g["atol"])
        s1 = api.Solution(p1, api.Launch(block=64, ckpt_every=1, ckpt_capacity=cap1))
        ms_f1 = timed(lambda: s1.run(), 3, 1, torch)
        yb1 = torch.ones((1, 6, 1), dtype=torch.float64, device="cuda")
        ms_v1 = timed(lambda: api.solve_vjp(s1, ybar_final=yb1), 3, 1, torch)
        vjp_roofline["critical_path"] = {
            "max_accepted_one_orbit": int(fused.n_accepted.max()),
            "longest_alone_ms": {"forward_with_tape": round(ms_f1, 3), "adjoint": round(ms_v1, 3)},
            "batch_adjoint_over_longest_alone": round(ms_vjp / ms_v1, 3)}
        log(f"[bench] adjoint kernel alone: {ms_vjp:.3f} ms, {ach_vjp:.2f} TFLOP/s "
            f"({100 * ach_vjp / PEAK_FP64_VECTOR_TFLOPS:.1f}% of FP64 peak); longest orbit alone "
            f"{ms_v1:.3f} ms")
        # The adjoint with the chip full: 10^6 orbits (t = 20, Dopri5 1e-8), store-mode tape.
        nv = 1_000_000
        vw = inputs.orbits_uneven(n=nv, seed=6)
        vp = api.make_problem(vw["rhs"], "dopri5", vw["y0"], vw["theta"], 0.0, np.full(nv, 20.0),
                              np.full(nv, 1e-8), np.full(nv, 1e-8))
        vplain = api.solve(vp, api.Launch(block=128))
        torch.cuda.synchronize()
        vcap = int(vplain.n_accepted.max()) + 2
        del vplain
        vsol = api.Solution(vp, api.Launch(block=128, ckpt_every=1, ckpt_capacity=vcap))
        vsol.run()
        vyb = vsol.y_final.clone().unsqueeze(0)
        vsteps = int(vsol.n_accepted.to(torch.int64).sum())
        ms_vf = timed(lambda: api.solve_vjp(vsol, ybar_final=vyb), 3, 1, torch)
        ach_vf = vsteps * fvs / (ms_vf * 1e-3) / 1e12
        vjp_roofline["full_chip"] = {
            "workload": "1,000,000 orbits, t = 20, Dopri5 rtol = atol = 1e-8, store-mode tape",
            "accepted_steps": vsteps, "ms": round(ms_vf, 4), "achieved": round(ach_vf, 3),
            "frac": round(ach_vf / PEAK_FP64_VECTOR_TFLOPS, 4)}
        log(f"[bench] adjoint kernel, chip full: {ms_vf:.3f} ms, {ach_vf:.2f} TFLOP/s "
            f"({100 * ach_vf / PEAK_FP64_VECTOR_TFLOPS:.1f}%)")
        del vsol, vyb
        torch.cuda.empty_cache()
        out["grad"] = {"workload": "orbits_gradient_100k", "ms_forward": round(ms_fwd, 4),
                       "forward_launch": {k: flaunch.__dict__[k]
                                          for k in ("block", "grid", "refill", "wide")},
                       "gradient_launch": gshape, "ms_gradient_by_launch": by_shape,
                       "ms_forward_in_gradient_launch": round(ms_fwd_same, 4),
                       "grad_forward_ratio_same_launch": round(best[1] / ms_fwd_same, 3),
                       "vjp_roofline": vjp_roofline,
                       "ms_forward_tape_plus_vjp": round(best[1], 4), "ckpt_every": best[0],
                       "ms_by_ckpt_every": per_k,
                       "arms_ms": {"fused_persistent_store_tape": round(ms_fused, 4),
                                   "one_lane_per_trajectory_store_tape": round(ms_stat, 4),
                                   "identical_gradients": same}}
        del fused, stat
        # The same two arms on the uneven batch (lengths spread over two decades), where a
        # wavefront of the plain arm waits for its longest trajectory in both passes.
        nu = prob.n
        cap_u = max_att // 32 + 2
        ybu = torch.zeros((1, 6, nu), dtype=torch.float64, device="cuda")
        Tu = torch.as_tensor(np.random.default_rng(8).normal(size=(3, nu)), device="cuda")
        ugrads = {}

        def ugrad_of(sol, grid):
            def step():
                sol.run()
                ybu[0, :3] = 2.0 * (sol.y_final[:3] - Tu)
                ugrads[grid] = api.solve_vjp(sol, ybar_final=ybu, grid=grid)
            return step

        ufused = api.Solution(prob, api.Launch(block=256, ckpt_every=32, ckpt_capacity=cap_u))
        ufused.set_order(order)
        ustat = api.Solution(prob, api.Launch(schedule="static", block=256, ckpt_every=32,
                                              ckpt_capacity=cap_u))
        ms_uf = timed(ugrad_of(ufused, 0), 3, 1, torch)
        ms_us = timed(ugrad_of(ustat, (nu + 255) // 256), 3, 1, torch)
        usame = all(torch.equal(a, b) for a, b in zip(ugrads[0], ugrads[(nu + 255) // 256]))
        log(f"[bench] uneven-batch gradient arms (k = 32): fused persistent {ms_uf:.3f} ms, one "
            f"lane per trajectory {ms_us:.3f} ms, identical gradients {usame}")
        out["grad"]["uneven_batch_arms_ms"] = {
            "workload": f"{nu} uneven orbits, checkpoints every 32 accepted steps, loss "
                        "sum |x(t1) - T|^2",
            "fused_persistent_longest_first": round(ms_uf, 4),
            "one_lane_per_trajectory": round(ms_us, 4), "identical_gradients": usame}
        del ufused, ustat
        out["grad_forward_ratio"] = best[1] / ms_fwd
        # The paper's own derivative: forward sensitivities in the same launch,
        # two columns (v0, q) as in its stream gradients, and all nine inputs
        # (longest first; the ratio is to the best forward).
        sens = {}
        for cols in ([6, 7], list(range(9))):
            ms_s = timed(lambda: api.solve_sens(pg, cols, order=gorder), max(3, args.steps // 4),
                         1, torch)
            sens[str(len(cols))] = {"ms": round(ms_s, 4), "ratio": round(ms_s / ms_fwd, 3)}
        out["grad"]["forward_sensitivities_by_columns"] = sens
        log(f"[bench] forward sensitivities: {sens}")

    # ---- dark-energy profile likelihood: 100 mocks x 100 slopes --------------------------
    if not args.no_grad:
        wd = inputs.de_profile_mocks()
        f = wd["fid"]
        kw = dict(newton=wd["newton"], mu=wd["mu"], trust=wd["trust"], rtol=wd["rtol"],
                  atol=wd["atol"], N_start=wd["t0"])
        # the solver's output nodes are the 64 dense redshifts; the model at the 7 data
        # redshifts comes from the spline through them
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
                            f"{wd['iters']} iterations, 64 solver nodes, spline to 7 data "
                            "redshifts"}
        # "a0 supplied": the flat amplitude at the start is handed in and moved to first order
        # with da0/dOm (no shooting in the timed fits)
        a0_flat = api.de_profile(lam, om0, h0, a00, wd["omega_r"], Nn, data, sigma, iters=0,
                                 **kw)["a0"]
        for name, newton, a0s in (("a0_solved", wd["newton"], a00), ("a0_supplied", 0, a0_flat)):
            def profile():
                return api.de_profile(lam, om0, h0, a0s, wd["omega_r"], Nn, data, sigma,
                                      iters=wd["iters"], **dict(kw, newton=newton))

            ms_p = timed(profile, max(3, args.steps // 4), 1, torch)
            res = profile()
            torch.cuda.synchronize()
            conv = ((res["chi2_prev"] - res["chi2"]).abs() < 1e-4) & \
                (res["decrement"].abs() < 1e-6)
            us_it = ms_p * 1e3 / (nfit * wd["iters"])
            prof[name] = {"newton_steps": newton, "ms": round(ms_p, 4),
                          "us_per_iteration_per_fit": round(us_it, 4),
                          "converged_fraction": round(float(conv.float().mean()), 4),
                          "all_ok": bool((res["status"] == 0).all())}
            log(f"[bench] dark-energy profile ({name}): {ms_p:.3f} ms, "
                f"{us_it:.4f} us per iteration per fit")
        out["de_profile"] = prof

    # ---- stiff path: Rodas4 on 10^5 trajectories of each kinetics network --------------------
    if not args.no_grad:
        out["stiff"] = stiff_bench(args, torch, api, inputs, autotune)

    # ---- the precession configuration at full size: the chip full for seconds --------------
    if not args.no_grad:
        out["roofline_showcase"] = precession_showcase(torch, api, inputs, autotune)
        out["precession_gradient"] = precession_gradient(torch, api, inputs)

    # ---- the paper's own per-trajectory workloads at 10^6 (its H200 figures as context) -------
    if not args.no_grad:
        out["paper_workloads"] = paper_workloads(torch, api, inputs, autotune)

    if not args.no_cpu:
        cb = cpu_baseline(w)
        out["cpu_baseline"] = cb
        log(f"[bench] cpu oracle: {cb['value']:.1f} solves/s on {cb['cores']} threads")

    print(json.dumps(out), flush=True)
    graph.close()


if __name__ == "__main__":
    main()
