"""Launch-shape autotuner for the ensemble solver.

For a problem class (right-hand side, tableau, log2 of the ensemble size,
device) it times candidate launch shapes of the forward kernel -- lanes per
workgroup, persistent-grid size (one or two wavefronts per SIMD, or the full
occupancy limit), refill granularity of the work queue, how many trajectories
at the head of a longest-first order run on 16-lane groups -- and, for gradient
runs, the checkpoint interval k of the tape (forward with tape plus adjoint).
The fastest shape is cached in a JSON file keyed by problem class.  Timing
uses HIP events on the stream the kernels run on.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import torch

from . import api

CACHE = os.environ.get("GS_AUTOTUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "gradsolve_autotune.json"))

BLOCKS = (64, 128, 256)
REFILLS = (1, 4, 8, 16, 64)
# Trajectories at the head of the queue order run on 16-lane groups (wide):
# tried on the best shapes when the call allows it (queue schedule, at most
# 16 state components, an explicit pair).
WIDES = (256, 512, 1024, 2048, 4096)
CKPT = (1, 8, 32, 128)  # 1 = store mode: every accepted step on the tape


def _key(prob: api.Problem, kind: str, base: api.Launch, ordered: bool) -> str:
    """Problem class of a cached shape: device, kind of run, right-hand side,
    tableau, log2 n, whether there are output nodes, the tape mode, whether a
    queue order is given, and the decades of the median span and tolerance
    (which set the step counts, so the tape sizes and the best shapes)."""
    dev = torch.cuda.get_device_name(prob.y0.device)
    span = float((prob.t1 - prob.t0).median()) if prob.n else 0.0
    rtol = float(prob.rtol.median()) if prob.n else 1.0
    return (f"{dev}|{kind}|rhs{prob.rhs}|tab{prob.tableau}|n2^{int(math.log2(max(prob.n, 1)))}"
            f"|K{int(prob.K > 0)}|ck{base.ckpt_every}|ord{int(ordered)}"
            f"|span10^{round(math.log10(max(span, 1e-300)))}"
            f"|rtol10^{round(math.log10(max(rtol, 1e-300)))}")


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(cache):
    os.makedirs(os.path.dirname(CACHE), exist_ok=True)
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def _time(fn, reps=3):
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def _grids(prob: api.Problem, block: int):
    cus = torch.cuda.get_device_properties(prob.y0.device).multi_processor_count
    waves_per_block = block // 64
    # one and two wavefronts per SIMD (4 SIMDs per CU), and the occupancy limit
    return sorted({max(1, (4 * cus) // waves_per_block), max(1, (8 * cus) // waves_per_block), 0})


def tune_forward(prob: api.Problem, order=None, base: api.Launch | None = None,
                 use_cache=True) -> api.Launch:
    """Fastest forward launch shape for this problem class."""
    base = base or api.Launch()
    key = _key(prob, "fwd", base, order is not None)
    cache = _load() if use_cache else {}
    if key in cache:
        return api.Launch(**{**base.__dict__, **cache[key]["launch"]})
    # Stage 1: every candidate, best of three.  Stage 2: the four fastest
    # again, seven times each in turn, ranked by the median (shapes within a
    # few percent of each other are otherwise picked by noise).
    scored = []
    for block in BLOCKS:
        for grid in _grids(prob, block):
            for refill in REFILLS:
                shape = {"schedule": "queue", "block": block, "grid": grid, "refill": refill,
                         "wide": 0}
                sol = api.Solution(prob, api.Launch(**{**base.__dict__, **shape}))
                if order is not None:
                    sol.set_order(order)
                scored.append((_time(lambda: sol.run()), shape))
    scored.sort(key=lambda x: x[0])
    if order is not None and prob.d <= 16 and prob.tableau != api.TABLEAU["rodas4"]:
        for _, shape0 in scored[:3]:
            for wide in WIDES:
                if wide >= prob.n:
                    continue
                shape = {**shape0, "wide": wide}
                sol = api.Solution(prob, api.Launch(**{**base.__dict__, **shape}))
                sol.set_order(order)
                scored.append((_time(lambda: sol.run()), shape))
        scored.sort(key=lambda x: x[0])
    finalists = []
    for _, shape in scored[:4]:
        sol = api.Solution(prob, api.Launch(**{**base.__dict__, **shape}))
        if order is not None:
            sol.set_order(order)
        finalists.append((sol, shape, []))
    for _ in range(7):
        for sol, _, times in finalists:
            times.append(_time(lambda: sol.run(), reps=1))
    best = min(((sorted(ts)[len(ts) // 2], shape) for _, shape, ts in finalists),
               key=lambda x: x[0])
    cache[key] = {"ms": best[0], "launch": best[1]}
    if use_cache:
        _store(cache)
    return api.Launch(**{**base.__dict__, **best[1]})


def _subset(prob: api.Problem, idx: torch.Tensor) -> api.Problem:
    """The trajectories idx of prob.  Per-trajectory arrays are sliced and shared
    ones kept, by their role: y0 [d][n]; theta [p][n] or shared [p]; t0, t1,
    rtol, atol [n] or shared [1]; t_out [K][n] or shared [K]."""
    def per_traj_2d(t):
        return None if t is None else (t[:, idx].contiguous() if t.dim() == 2 else t)

    def per_traj_1d(t):
        return t[idx].contiguous() if t.numel() == prob.n and t.numel() > 1 else t
    return api.Problem(prob.rhs, prob.tableau, per_traj_2d(prob.y0), per_traj_2d(prob.theta),
                       per_traj_1d(prob.t0), per_traj_1d(prob.t1), per_traj_1d(prob.rtol),
                       per_traj_1d(prob.atol), per_traj_2d(prob.t_out))


def pilot_order(prob: api.Problem, features, sample: int = 4096,
                launch: api.Launch | None = None, seed: int = 0):
    """Longest-first queue order from a pilot solve, for ensembles whose cost
    has no closed-form model: a random sample of the trajectories is solved,
    their step attempts are fitted by least squares on the features ([F][n]
    host arrays, e.g. logarithms of parameters and spans), and every
    trajectory is ordered by its fitted cost, largest first.  The pilot is
    set-up work, like the launch-shape search."""
    n = prob.n
    feats = [np.asarray(f, float).reshape(-1) for f in features]
    if any(f.shape != (n,) or not np.all(np.isfinite(f)) for f in feats):
        raise ValueError("features must be finite arrays of one value per trajectory")
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(n, min(sample, n), replace=False))
    sub = _subset(prob, torch.as_tensor(idx, device=prob.y0.device))
    sol = api.solve(sub, launch or api.Launch())
    att = (sol.n_accepted + sol.n_rejected).double().cpu().numpy()
    F = np.column_stack([np.ones(n)] + feats)
    coef, *_ = np.linalg.lstsq(F[idx], att, rcond=None)
    return np.argsort(-(F @ coef), kind="stable").astype(np.int64)


def pilot_cost(prob: api.Problem, features: torch.Tensor, sample: int = 4096,
               launch: api.Launch | None = None, seed: int = 0,
               tol_scale: float = 1.0) -> torch.Tensor:
    """Fitted cost of every trajectory on the device, for gs_queue_order
    (``Solution.queue_order(cost)``): a pilot solve of a random sample of the
    trajectories, a least-squares fit of their step attempts on the features
    (a device tensor [F][n]) plus a constant, and the fitted attempts of all
    n.  ``tol_scale`` > 1 runs the pilot at looser tolerances (the ranking of
    the costs, not their size, sets the order, and a pilot's time is that of
    its longest trajectory).  The pilot and the fit are part of building the
    order; callers that time the ensemble report them."""
    n = prob.n
    dev = prob.y0.device
    F = torch.cat([torch.ones((1, n), dtype=torch.float64, device=dev),
                   features.to(device=dev, dtype=torch.float64)]).T.contiguous()  # [n][1+F]
    g = torch.Generator(device="cpu").manual_seed(seed)
    idx = torch.randperm(n, generator=g)[:min(sample, n)].sort().values.to(dev)
    sub = _subset(prob, idx)
    sub.t_out = None  # output times do not change the steps
    if tol_scale != 1.0:
        sub.rtol, sub.atol = sub.rtol * tol_scale, sub.atol * tol_scale
    sol = api.solve(sub, launch or api.Launch())
    att = (sol.n_accepted + sol.n_rejected).to(torch.float64)
    coef = torch.linalg.lstsq(F[idx].cpu(), att.cpu().unsqueeze(1)).solution
    return (F @ coef.to(dev)).reshape(n)


def tune_gradient(prob: api.Problem, make_cotangent, base: api.Launch | None = None,
                  use_cache=True, order=None) -> api.Launch:
    """Fastest launch for forward-with-tape plus adjoint: the checkpoint
    interval k, and the launch shape of both passes (the base shape, two
    waves per CU, one wave per SIMD; with a queue order also the head of
    the order on 16-lane groups in the forward).  Run the adjoint
    with the returned block and grid (``solve_vjp(..., block=, grid=)``).

    ``make_cotangent(sol)`` returns (ybar_final, ybar_out) for a solution.
    """
    base = base or api.Launch()
    key = _key(prob, "grad", base, order is not None)
    cache = _load() if use_cache else {}
    # The tape capacity is sized for this problem from a plain solve, never
    # taken from the cache (a problem of the same class may take more steps).
    plain = api.solve(prob, api.Launch(**{**base.__dict__, "ckpt_every": 0, "wide": 0}))
    torch.cuda.synchronize()
    nmax = int(plain.n_accepted.max())
    del plain
    if key in cache:
        shape = dict(cache[key]["launch"])
        shape["ckpt_capacity"] = nmax // shape["ckpt_every"] + 2
        return api.Launch(**{**base.__dict__, **shape})
    cus = torch.cuda.get_device_properties(prob.y0.device).multi_processor_count
    shapes = [(base.block, base.grid, 0), (128, 2 * cus, 0), (64, 4 * cus, 0)]
    if order is not None and prob.d <= 16 and prob.tableau != api.TABLEAU["rodas4"]:
        shapes.append((128, 2 * cus, 256))
    best = None
    free = torch.cuda.mem_get_info(prob.y0.device)[0]
    for block, grid, wide in shapes:
        for k in CKPT:
            shape = {"block": block, "grid": grid, "wide": wide, "ckpt_every": k,
                     "ckpt_capacity": nmax // k + 2}
            L = api.Launch(**{**base.__dict__, **shape})
            if api.workspace_bytes(prob, L) > free // 2:
                continue  # the tape would crowd out everything else
            sol = api.Solution(prob, L)
            if order is not None:
                sol.set_order(order)

            def step():
                sol.run()
                yf, yo = make_cotangent(sol)
                api.solve_vjp(sol, ybar_final=yf, ybar_out=yo, block=block, grid=grid)

            ms = _time(step)
            if best is None or ms < best[0]:
                best = (ms, shape)
            del sol
    cache[key] = {"ms": best[0], "launch": {k: v for k, v in best[1].items()
                                            if k != "ckpt_capacity"}}
    if use_cache:
        _store(cache)
    return api.Launch(**{**base.__dict__, **best[1]})
