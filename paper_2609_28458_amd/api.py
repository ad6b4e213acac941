"""Thin binding of the C ABI in ``include/gradsolve.h`` (ctypes).

Argument marshalling only: every step of the solve, its gradient and the
dense query runs in the HIP kernels of ``libgradsolve.so``.  torch supplies
device memory and the current stream.  The low-level functions carry the C
names (``gs_solve``, ``gs_solve_vjp``, ``gs_dense_eval``, ``gs_rhs_eval``,
``gs_workspace_bytes``, ``gs_graph_*``); ``solve``/``solve_vjp``/``dense_eval``
build the argument structs from torch tensors.

If the library is missing this module raises on first use: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgradsolve.so")

RHS = {"harmonic": 0, "kepler": 1, "loghalo": 2, "spinprec": 3, "quint": 4, "kin3": 5,
       "kin8": 6, "rober": 7, "hires": 8}
DIM = {0: 2, 1: 4, 2: 6, 3: 9, 4: 3, 5: 3, 6: 8, 7: 3, 8: 8}
NPARAM = {0: 1, 1: 1, 2: 3, 3: 3, 4: 4, 5: 3, 6: 12, 7: 3, 8: 8}
TABLEAU = {"dopri5": 0, "tsit5": 1, "verner7": 2, "rodas4": 3}
SCHEDULE = {"queue": 0, "static": 1}
OUT_LAYOUT = {"dkn": 0, "knd": 1}
TRAJ_STATUS = {0: "OK", 1: "MAX_STEPS", 2: "DT_UNDERFLOW", 3: "NONFINITE",
               4: "TAPE_OVERFLOW", 5: "BAD_INPUT", 6: "NOT_RUN"}
GS_OK = 0


class GsError(RuntimeError):
    pass


class gs_controller(C.Structure):
    _fields_ = [("safety", C.c_double), ("alpha_min", C.c_double), ("alpha_max", C.c_double),
                ("beta1", C.c_double), ("beta2", C.c_double)]


class gs_solve_args(C.Structure):
    _fields_ = [
        ("rhs", C.c_int32), ("tableau", C.c_int32), ("n", C.c_int64),
        ("d", C.c_int32), ("p", C.c_int32),
        ("y0", C.c_void_p), ("theta", C.c_void_p), ("theta_stride", C.c_int64),
        ("t0", C.c_void_p), ("t1", C.c_void_p), ("t_stride", C.c_int64),
        ("rtol", C.c_void_p), ("atol", C.c_void_p), ("tol_stride", C.c_int64),
        ("K", C.c_int32), ("t_out", C.c_void_p), ("t_out_stride", C.c_int64),
        ("y_out", C.c_void_p), ("y_final", C.c_void_p),
        ("n_accepted", C.c_void_p), ("n_rejected", C.c_void_p), ("status", C.c_void_p),
        ("max_steps", C.c_int64), ("h0", C.c_double), ("ctrl", gs_controller),
        ("ckpt_every", C.c_int32), ("ckpt_capacity", C.c_int32),
        ("schedule", C.c_int32), ("block", C.c_int32), ("grid", C.c_int32),
        ("refill", C.c_int32), ("wide", C.c_int32), ("order", C.c_void_p),
        ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t), ("stream", C.c_void_p),
        ("out_layout", C.c_int32),
    ]


class gs_vjp_args(C.Structure):
    _fields_ = [
        ("R", C.c_int32), ("ybar_out", C.c_void_p), ("ybar_final", C.c_void_p),
        ("y0bar", C.c_void_p), ("thetabar", C.c_void_p), ("block", C.c_int32),
        ("grid", C.c_int32), ("stream", C.c_void_p), ("wide", C.c_int32),
    ]


class gs_sens_args(C.Structure):
    _fields_ = [
        ("M", C.c_int32), ("cols", C.c_void_p), ("S_final", C.c_void_p), ("S_out", C.c_void_p),
    ]


class gs_de_profile_args(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("lambda_", C.c_void_p), ("omega_m", C.c_void_p), ("h", C.c_void_p),
        ("a0", C.c_void_p), ("omega_r", C.c_double), ("K", C.c_int32), ("N_nodes", C.c_void_p),
        ("K_data", C.c_int32), ("N_data", C.c_void_p), ("data", C.c_void_p), ("sigma", C.c_void_p), ("iters", C.c_int32), ("newton", C.c_int32),
        ("mu", C.c_double), ("trust_om", C.c_double), ("trust_h", C.c_double),
        ("tableau", C.c_int32), ("N_start", C.c_double), ("rtol", C.c_double),
        ("atol", C.c_double), ("chi2", C.c_void_p), ("chi2_prev", C.c_void_p),
        ("decrement", C.c_void_p), ("dist", C.c_void_p), ("status", C.c_void_p),
        ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t), ("stream", C.c_void_p),
    ]


EXPORTS = ["gs_default_args", "gs_workspace_bytes", "gs_solve", "gs_solve_noalloc",
           "gs_queue_order", "gs_queue_order_workspace_bytes", "gs_solve_vjp", "gs_solve_sens",
           "gs_de_profile", "gs_de_profile_workspace_bytes", "gs_dense_eval",
           "gs_rhs_eval", "gs_graph_create", "gs_graph_launch", "gs_graph_destroy",
           "gs_status_string", "gs_version"]

_lib = None


def lib():
    """Load libgradsolve.so (built in-tree by ``build.build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise GsError(f"{LIB_PATH} is missing: build it with "
                          "paper_2609_28458_amd.build.build() (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        L.gs_default_args.argtypes = [C.POINTER(gs_solve_args)]
        L.gs_default_args.restype = None
        L.gs_workspace_bytes.argtypes = [C.POINTER(gs_solve_args)]
        L.gs_workspace_bytes.restype = C.c_size_t
        L.gs_solve.argtypes = [C.POINTER(gs_solve_args)]
        L.gs_solve.restype = C.c_int
        L.gs_solve_noalloc.argtypes = [C.POINTER(gs_solve_args)]
        L.gs_solve_noalloc.restype = C.c_int
        L.gs_queue_order.argtypes = [C.POINTER(gs_solve_args), C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_size_t]
        L.gs_queue_order.restype = C.c_int
        L.gs_queue_order_workspace_bytes.argtypes = [C.c_int64]
        L.gs_queue_order_workspace_bytes.restype = C.c_size_t
        L.gs_solve_vjp.argtypes = [C.POINTER(gs_solve_args), C.POINTER(gs_vjp_args)]
        L.gs_solve_vjp.restype = C.c_int
        L.gs_solve_sens.argtypes = [C.POINTER(gs_solve_args), C.POINTER(gs_sens_args)]
        L.gs_solve_sens.restype = C.c_int
        L.gs_de_profile.argtypes = [C.POINTER(gs_de_profile_args)]
        L.gs_de_profile.restype = C.c_int
        L.gs_de_profile_workspace_bytes.argtypes = [C.POINTER(gs_de_profile_args)]
        L.gs_de_profile_workspace_bytes.restype = C.c_size_t
        L.gs_dense_eval.argtypes = [C.POINTER(gs_solve_args), C.c_int32, C.c_void_p, C.c_void_p,
                                    C.c_void_p]
        L.gs_dense_eval.restype = C.c_int
        L.gs_rhs_eval.argtypes = [C.c_int32, C.c_int64] + [C.c_void_p] * 8
        L.gs_rhs_eval.restype = C.c_int
        L.gs_graph_create.argtypes = [C.POINTER(gs_solve_args), C.POINTER(C.c_void_p)]
        L.gs_graph_create.restype = C.c_int
        L.gs_graph_launch.argtypes = [C.c_void_p, C.c_void_p]
        L.gs_graph_launch.restype = C.c_int
        L.gs_graph_destroy.argtypes = [C.c_void_p]
        L.gs_graph_destroy.restype = None
        L.gs_status_string.argtypes = [C.c_int]
        L.gs_status_string.restype = C.c_char_p
        L.gs_version.argtypes = []
        L.gs_version.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != GS_OK:
        raise GsError(f"gradsolve: {lib().gs_status_string(rc).decode()} (code {rc})")


# ----- the C entry points under their own names ---------------------------------------------

def gs_default_args() -> gs_solve_args:
    a = gs_solve_args()
    lib().gs_default_args(C.byref(a))
    return a


def gs_workspace_bytes(args: gs_solve_args) -> int:
    return int(lib().gs_workspace_bytes(C.byref(args)))


def gs_solve(args: gs_solve_args) -> None:
    _check(lib().gs_solve(C.byref(args)))


def gs_solve_noalloc(args: gs_solve_args) -> None:
    _check(lib().gs_solve_noalloc(C.byref(args)))


def gs_queue_order(args: gs_solve_args, cost: int | None, order: int, workspace: int,
                   workspace_bytes: int) -> None:
    _check(lib().gs_queue_order(C.byref(args), cost, order, workspace, workspace_bytes))


def gs_queue_order_workspace_bytes(n: int) -> int:
    return int(lib().gs_queue_order_workspace_bytes(n))


def gs_solve_vjp(args: gs_solve_args, vjp: gs_vjp_args) -> None:
    _check(lib().gs_solve_vjp(C.byref(args), C.byref(vjp)))


def gs_dense_eval(args: gs_solve_args, Q: int, t_query: int, y_query: int, stream: int) -> None:
    _check(lib().gs_dense_eval(C.byref(args), Q, t_query, y_query, stream))


def gs_rhs_eval(rhs, m, t, y, theta, f, kbar, ybar, thetabar, stream) -> None:
    _check(lib().gs_rhs_eval(rhs, m, t, y, theta, f, kbar, ybar, thetabar, stream))


def gs_graph_create(args: gs_solve_args) -> int:
    h = C.c_void_p()
    _check(lib().gs_graph_create(C.byref(args), C.byref(h)))
    return h.value


def gs_graph_launch(handle: int, stream: int) -> None:
    _check(lib().gs_graph_launch(handle, stream))


def gs_graph_destroy(handle: int) -> None:
    lib().gs_graph_destroy(handle)


def gs_version() -> str:
    return lib().gs_version().decode()


# ----- torch-facing helpers ------------------------------------------------------------------

def _ptr(t):
    return None if t is None else t.data_ptr()


def _dev(x, device, dtype=torch.float64):
    if isinstance(x, torch.Tensor):
        t = x.to(device=device, dtype=dtype)
    else:
        t = torch.as_tensor(x, dtype=dtype, device=device)
    return t.contiguous()


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


@dataclass
class Problem:
    """Device-resident inputs of an ensemble solve (SoA layouts of the C ABI)."""
    rhs: int
    tableau: int
    y0: torch.Tensor            # [d][n]
    theta: torch.Tensor         # [p] or [p][n]
    t0: torch.Tensor            # [1] or [n]
    t1: torch.Tensor
    rtol: torch.Tensor
    atol: torch.Tensor
    t_out: torch.Tensor | None  # [K] or [K][n]

    @property
    def n(self):
        return self.y0.shape[1]

    @property
    def d(self):
        return self.y0.shape[0]

    @property
    def K(self):
        return 0 if self.t_out is None else self.t_out.shape[0]


def make_problem(rhs, tableau, y0, theta, t0, t1, rtol, atol, t_out=None, device="cuda"):
    rid = RHS[rhs] if isinstance(rhs, str) else int(rhs)
    tid = TABLEAU[tableau] if isinstance(tableau, str) else int(tableau)
    y0 = _dev(y0, device)
    d, n = y0.shape
    if d != DIM[rid]:
        raise ValueError(f"y0 must have {DIM[rid]} rows")
    th = _dev(theta, device)
    if th.dim() == 2 and th.shape != (NPARAM[rid], n):
        raise ValueError("theta must be [p] or [p][n]")
    if th.dim() == 1 and th.shape[0] != NPARAM[rid]:
        raise ValueError("theta must be [p] or [p][n]")

    def scal(x):
        t = _dev(x, device).reshape(-1)
        if t.numel() not in (1, n):
            raise ValueError("per-trajectory values must be scalars or [n]")
        return t

    t0t, t1t = scal(t0), scal(t1)
    if t0t.numel() != t1t.numel():
        t0t, t1t = t0t.expand(n).contiguous(), t1t.expand(n).contiguous()
    rt, at = scal(rtol), scal(atol)
    if rt.numel() != at.numel():
        rt, at = rt.expand(n).contiguous(), at.expand(n).contiguous()
    to = None if t_out is None else _dev(t_out, device)
    return Problem(rid, tid, y0, th, t0t, t1t, rt, at, to)


@dataclass
class Launch:
    schedule: str = "queue"
    block: int = 0
    grid: int = 0
    refill: int = 0
    wide: int = 0
    ckpt_every: int = 0
    ckpt_capacity: int = 0
    max_steps: int = 0
    h0: float = 0.0
    safety: float = 0.9
    alpha_min: float = 0.2
    alpha_max: float = 5.0
    beta1: float = 0.0
    beta2: float = 0.0
    out_layout: str = "dkn"  # y_out [d][K][n]; "knd": [K][n][d]


def workspace_bytes(prob: Problem, launch: Launch) -> int:
    """Device workspace a solve of `prob` with `launch` needs (gs_workspace_bytes)."""
    a = gs_default_args()
    a.rhs, a.tableau, a.n, a.d, a.p = prob.rhs, prob.tableau, prob.n, prob.d, NPARAM[prob.rhs]
    a.ckpt_every, a.ckpt_capacity = launch.ckpt_every, launch.ckpt_capacity
    a.K = prob.K
    return gs_workspace_bytes(a)


class Solution:
    """Outputs and the buffers a later gradient or dense query reads."""

    def __init__(self, prob: Problem, launch: Launch):
        dev = prob.y0.device
        n, d, K = prob.n, prob.d, prob.K
        self.prob = prob
        self.launch = launch
        shape = (K, n, d) if launch.out_layout == "knd" else (d, K, n)
        self.y_out = torch.empty(shape, dtype=torch.float64, device=dev) if K else None
        self.y_final = torch.empty((d, n), dtype=torch.float64, device=dev)
        self.n_accepted = torch.empty(n, dtype=torch.int32, device=dev)
        self.n_rejected = torch.empty(n, dtype=torch.int32, device=dev)
        self.status = torch.empty(n, dtype=torch.int32, device=dev)
        self.order = None
        self.args = self._args()
        nbytes = gs_workspace_bytes(self.args)
        # 256-byte alignment is guaranteed by torch's caching allocator.
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
        self.args.workspace = self.workspace.data_ptr()
        self.args.workspace_bytes = self.workspace.numel()

    def _args(self):
        p, L = self.prob, self.launch
        a = gs_default_args()
        a.rhs, a.tableau, a.n, a.d, a.p = p.rhs, p.tableau, p.n, p.d, NPARAM[p.rhs]
        a.y0 = _ptr(p.y0)
        a.theta = _ptr(p.theta)
        a.theta_stride = 0 if p.theta.dim() == 1 else p.n
        a.t0, a.t1 = _ptr(p.t0), _ptr(p.t1)
        a.t_stride = 0 if p.t0.numel() == 1 else 1
        a.rtol, a.atol = _ptr(p.rtol), _ptr(p.atol)
        a.tol_stride = 0 if p.rtol.numel() == 1 else 1
        a.K = p.K
        a.t_out = _ptr(p.t_out)
        a.t_out_stride = 0 if (p.t_out is None or p.t_out.dim() == 1) else p.n
        a.y_out = _ptr(self.y_out)
        a.y_final = _ptr(self.y_final)
        a.n_accepted, a.n_rejected, a.status = (_ptr(self.n_accepted), _ptr(self.n_rejected),
                                                _ptr(self.status))
        a.max_steps = L.max_steps
        a.h0 = L.h0
        a.ctrl = gs_controller(L.safety, L.alpha_min, L.alpha_max, L.beta1, L.beta2)
        a.ckpt_every, a.ckpt_capacity = L.ckpt_every, L.ckpt_capacity
        a.schedule = SCHEDULE[L.schedule]
        a.block, a.grid, a.refill, a.wide = L.block, L.grid, L.refill, L.wide
        a.out_layout = OUT_LAYOUT[L.out_layout]
        return a

    def set_order(self, order, check=True):
        """Queue order of the trajectories (longest first, say), a permutation
        of 0..n-1.  With ``check`` it is verified to be one (a device sort and
        one host synchronisation); the library itself marks any index an order
        misses as NOT_RUN."""
        self.order = None if order is None else _dev(order, self.prob.y0.device, torch.int64)
        if self.order is not None and check:
            n = self.prob.n
            ok = self.order.shape == (n,) and bool(torch.equal(
                torch.sort(self.order).values,
                torch.arange(n, dtype=torch.int64, device=self.order.device)))
            if not ok:
                raise ValueError("order must be a permutation of 0..n-1")
        self.args.order = _ptr(self.order)

    def queue_order(self, cost=None, stream=None):
        """Build a longest-first order on the device (gs_queue_order) into this
        solution's order buffer and use it: the library's cost model, or
        ``cost`` [n] (larger first).  Asynchronous; returns the order tensor."""
        dev = self.prob.y0.device
        n = self.prob.n
        if self.order is None or self.order.shape != (n,):
            self.order = torch.empty(n, dtype=torch.int64, device=dev)
        nb = gs_queue_order_workspace_bytes(n)
        if getattr(self, "_order_ws", None) is None or self._order_ws.numel() < nb:
            self._order_ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
        self._order_cost = None if cost is None else _dev(cost, dev).reshape(n)
        self.args.stream = _stream_handle(stream)
        gs_queue_order(self.args, _ptr(self._order_cost), _ptr(self.order),
                       self._order_ws.data_ptr(), self._order_ws.numel())
        self.args.order = _ptr(self.order)
        return self.order

    def run_noalloc(self, stream=None):
        """The same solve through gs_solve_noalloc (no tape; the library's static
        scratch instead of this solution's workspace)."""
        self.args.stream = _stream_handle(stream)
        gs_solve_noalloc(self.args)
        return self

    def run(self, stream=None):
        self.args.stream = _stream_handle(stream)
        gs_solve(self.args)
        return self

    def replay_mismatches(self) -> int:
        """Adjoint segment replays that did not reproduce the next checkpoint."""
        return int(self.workspace[16:24].view(torch.int64).item())


def solve(prob: Problem, launch: Launch | None = None, order=None, stream=None) -> Solution:
    sol = Solution(prob, launch or Launch())
    if order is not None:
        sol.set_order(order)
    return sol.run(stream)


def gs_solve_sens(args: gs_solve_args, sens: gs_sens_args) -> None:
    _check(lib().gs_solve_sens(C.byref(args), C.byref(sens)))


def solve_sens(prob: Problem, cols, launch: Launch | None = None, stream=None, order=None):
    """Solution plus forward sensitivities (eq:sens) of the columns ``cols``:
    index c < d is y0[c], d + q is theta[q].  Returns (Solution, S_final
    [d][M][n], S_out [d][M][K][n] or None).  ``order``: queue order, as for
    solve."""
    sol = Solution(prob, launch or Launch())
    if order is not None:
        sol.set_order(order)
    cols = [int(c) for c in cols]
    M = len(cols)
    dev = prob.y0.device
    S_final = torch.empty((prob.d, M, prob.n), dtype=torch.float64, device=dev)
    S_out = (torch.empty((prob.d, M, prob.K, prob.n), dtype=torch.float64, device=dev)
             if prob.K else None)
    ccols = (C.c_int32 * M)(*cols)
    s = gs_sens_args(M, C.cast(ccols, C.c_void_p), _ptr(S_final), _ptr(S_out))
    sol.args.stream = _stream_handle(stream)
    gs_solve_sens(sol.args, s)
    return sol, S_final, S_out


def gs_de_profile(args: gs_de_profile_args) -> None:
    _check(lib().gs_de_profile(C.byref(args)))


def de_profile(lam, omega_m, h, a0, omega_r, N_nodes, data, sigma, *, iters=20, newton=3,
               mu=1e-3, trust=(0.05, 0.05), tableau="dopri5", N_start=None, rtol=1.78e-4,
               atol=1.78e-7, N_data=None, device="cuda", stream=None):
    """Dark-energy profile fits (gs_de_profile): n minimisations at fixed
    lam [n], psi = (omega_m, h) from the given starts, a0 [n] the starting
    amplitudes; data [2][Kd][n], sigma [2][Kd] at the K nodes (Kd = K) or,
    with N_data [Kd], at those e-folds through the spline over the nodes.
    Returns a dict of device tensors: omega_m, h, a0, chi2, chi2_prev,
    decrement, dist [2][Kd][n], status."""
    f64 = dict(dtype=torch.float64, device=device)
    lam_t = torch.as_tensor(lam, **f64).contiguous()
    n = lam_t.numel()
    out = {"omega_m": torch.as_tensor(omega_m, **f64).clone().contiguous(),
           "h": torch.as_tensor(h, **f64).clone().contiguous(),
           "a0": torch.as_tensor(a0, **f64).clone().contiguous()}
    Nn = torch.as_tensor(N_nodes, **f64).contiguous()
    K = Nn.numel()
    Nd = None if N_data is None else torch.as_tensor(N_data, **f64).contiguous()
    Kd = K if Nd is None else Nd.numel()
    data_t = torch.as_tensor(data, **f64).contiguous()
    sig_t = torch.as_tensor(sigma, **f64).contiguous()
    if tuple(data_t.shape) != (2, Kd, n) or tuple(sig_t.shape) != (2, Kd):
        raise ValueError("data must be [2][Kd][n] and sigma [2][Kd]")
    for k in ("chi2", "chi2_prev", "decrement"):
        out[k] = torch.empty(n, **f64)
    out["dist"] = torch.empty((2, Kd, n), **f64)
    out["status"] = torch.empty(n, dtype=torch.int32, device=device)
    a = gs_de_profile_args()
    a.n, a.lambda_, a.omega_m, a.h, a.a0 = n, _ptr(lam_t), _ptr(out["omega_m"]), _ptr(out["h"]), \
        _ptr(out["a0"])
    a.omega_r, a.K, a.N_nodes, a.data, a.sigma = float(omega_r), K, _ptr(Nn), _ptr(data_t), \
        _ptr(sig_t)
    a.K_data, a.N_data = (0, None) if Nd is None else (Kd, _ptr(Nd))
    a.iters, a.newton, a.mu = int(iters), int(newton), float(mu)
    a.trust_om, a.trust_h = float(trust[0]), float(trust[1])
    a.tableau = TABLEAU[tableau] if isinstance(tableau, str) else int(tableau)
    a.N_start = float(-np.log(51.0) if N_start is None else N_start)
    a.rtol, a.atol = float(rtol), float(atol)
    a.chi2, a.chi2_prev, a.decrement = _ptr(out["chi2"]), _ptr(out["chi2_prev"]), \
        _ptr(out["decrement"])
    a.dist, a.status = _ptr(out["dist"]), _ptr(out["status"])
    nbytes = int(lib().gs_de_profile_workspace_bytes(C.byref(a)))
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
    a.workspace, a.workspace_bytes = ws.data_ptr(), ws.numel()
    a.stream = _stream_handle(stream)
    gs_de_profile(a)
    out["_keep"] = (lam_t, Nn, Nd, data_t, sig_t, ws)
    return out


def solve_vjp(sol: Solution, ybar_final=None, ybar_out=None, block=0, grid=0, stream=None,
              wide=0):
    """Cotangents [R][d][n] / [R][d][K][n] -> (y0bar [R][d][n], thetabar [R][p][n]).
    ``wide``: the head of the queue order reversed on 16-lane groups (store-mode
    tape, final-state cotangents only)."""
    p = sol.prob
    dev = p.y0.device
    ref = ybar_final if ybar_final is not None else ybar_out
    if ref is None:
        raise ValueError("need ybar_final or ybar_out")
    R = ref.shape[0]
    yf = None if ybar_final is None else _dev(ybar_final, dev)
    yo = None if ybar_out is None else _dev(ybar_out, dev)
    if yf is not None and tuple(yf.shape) != (R, p.d, p.n):
        raise ValueError("ybar_final must be [R][d][n]")
    if yo is not None and tuple(yo.shape) != (R, p.d, p.K, p.n):
        raise ValueError("ybar_out must be [R][d][K][n]")
    y0bar = torch.empty((R, p.d, p.n), dtype=torch.float64, device=dev)
    thbar = torch.empty((R, NPARAM[p.rhs], p.n), dtype=torch.float64, device=dev)
    v = gs_vjp_args(R, _ptr(yo), _ptr(yf), _ptr(y0bar), _ptr(thbar), block, grid,
                    _stream_handle(stream), int(wide))
    sol.args.stream = v.stream
    gs_solve_vjp(sol.args, v)
    return y0bar, thbar


def dense_eval(sol: Solution, t_query, stream=None):
    """y at t_query [Q][n] -> [d][Q][n]."""
    p = sol.prob
    tq = _dev(t_query, p.y0.device)
    if tq.dim() != 2 or tq.shape[1] != p.n:
        raise ValueError("t_query must be [Q][n]")
    yq = torch.empty((p.d, tq.shape[0], p.n), dtype=torch.float64, device=p.y0.device)
    gs_dense_eval(sol.args, tq.shape[0], tq.data_ptr(), yq.data_ptr(), _stream_handle(stream))
    return yq


def rhs_eval(rhs, t, y, theta, kbar=None, stream=None):
    """Pointwise f and, with kbar, (J_y^T kbar, J_theta^T kbar); SoA [d][m] inputs."""
    rid = RHS[rhs] if isinstance(rhs, str) else int(rhs)
    y = _dev(y, "cuda")
    m = y.shape[1]
    t = _dev(t, "cuda").reshape(m)
    th = _dev(theta, "cuda")
    f = torch.empty_like(y)
    if kbar is None:
        gs_rhs_eval(rid, m, t.data_ptr(), y.data_ptr(), th.data_ptr(), f.data_ptr(), None, None,
                    None, _stream_handle(stream))
        return f
    kb = _dev(kbar, "cuda")
    yb = torch.empty_like(y)
    tb = torch.empty_like(th)
    gs_rhs_eval(rid, m, t.data_ptr(), y.data_ptr(), th.data_ptr(), f.data_ptr(), kb.data_ptr(),
                yb.data_ptr(), tb.data_ptr(), _stream_handle(stream))
    return f, yb, tb


class Captured:
    """Any sequence of library calls on one stream (say gs_queue_order then
    gs_solve) captured into one graph with torch.cuda.CUDAGraph and replayed
    with launch().  ``fn(stream)`` issues the calls on the stream it is
    given; the calls allocate nothing, so the graph holds only their kernels."""

    def __init__(self, fn):
        self.stream = torch.cuda.Stream()
        self.graph = torch.cuda.CUDAGraph()
        self.stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(self.graph, stream=self.stream, capture_error_mode="thread_local"):
            fn(self.stream)
        torch.cuda.current_stream().wait_stream(self.stream)

    def launch(self):
        self.graph.replay()


class Graph:
    """One gs_solve captured into a hipGraph; replay with launch()."""

    def __init__(self, sol: Solution):
        self.sol = sol
        self.handle = gs_graph_create(sol.args)

    def launch(self, stream=None):
        gs_graph_launch(self.handle, _stream_handle(stream))

    def close(self):
        if self.handle:
            gs_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
