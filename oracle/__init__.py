"""Oracle -- test infrastructure only.

A plain, slow FP64 CPU reference for the adaptive explicit Runge--Kutta
ensemble solve of the paper (Appendix "Numerical details": eq:rk,
eq:errnorm, eq:controller, eq:dense, eq:stage-sens), and for the stiff path:
a Rosenbrock solve (Rodas4 in the textbook form) of stiff kinetics networks
(``stiff.cpp``).  It is loaded only by
the test suite, the smoke check and the CPU-baseline leg of the benchmark; the
product library never imports it and shares no source with it.

The C++ sources sit beside this file and build into ``libgso.so``
(``g++ -O2 -fno-fast-math -ffp-contract=off``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgso.so")
SOURCES = ["solver.cpp", "tableaux.cpp", "stiff.cpp"]

RHS = {"harmonic": 0, "kepler": 1, "loghalo": 2, "spinprec": 3, "quint": 4, "kin3": 5,
       "kin8": 6, "rober": 7, "hires": 8}
DIM = {0: 2, 1: 4, 2: 6, 3: 9, 4: 3, 5: 3, 6: 8, 7: 3, 8: 8}
NPARAM = {0: 1, 1: 1, 2: 3, 3: 3, 4: 4, 5: 3, 6: 12, 7: 3, 8: 8}
TABLEAU = {"dopri5": 0, "tsit5": 1, "verner7": 2, "rodas4": 3}
STIFF_RHS = (5, 6, 7, 8)
STATUS = {0: "OK", 1: "MAX_STEPS", 2: "DT_UNDERFLOW", 3: "NONFINITE"}


def build(force: bool = False) -> str:
    """Compile the oracle into libgso.so next to the sources."""
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    hdrs = [os.path.join(HERE, h) for h in ("gso.hpp", "rhs.hpp", "dual.hpp")]
    if not force and os.path.exists(LIB_PATH):
        mt = os.path.getmtime(LIB_PATH)
        if all(os.path.getmtime(f) <= mt for f in srcs + hdrs):
            return LIB_PATH
    cmd = ["g++", "-O2", "-fno-fast-math", "-ffp-contract=off", "-std=c++17", "-shared",
           "-fPIC", "-o", LIB_PATH + ".tmp"] + srcs + ["-lpthread"]
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class _Problem(C.Structure):
    _fields_ = [
        ("rhs", C.c_int32), ("tableau", C.c_int32), ("n", C.c_int64),
        ("y0", C.c_void_p), ("theta", C.c_void_p), ("theta_stride", C.c_int64),
        ("t0", C.c_void_p), ("t1", C.c_void_p), ("t_stride", C.c_int64),
        ("rtol", C.c_void_p), ("atol", C.c_void_p), ("tol_stride", C.c_int64),
        ("K", C.c_int32), ("t_out", C.c_void_p), ("t_out_stride", C.c_int64),
        ("y_out", C.c_void_p), ("y_final", C.c_void_p),
        ("n_acc", C.c_void_p), ("n_rej", C.c_void_p), ("status", C.c_void_p),
        ("max_steps", C.c_int64), ("h0", C.c_double),
        ("safety", C.c_double), ("alpha_min", C.c_double), ("alpha_max", C.c_double),
        ("beta1", C.c_double), ("beta2", C.c_double),
        ("no_grow_after_reject", C.c_int32), ("nthreads", C.c_int32),
        ("m", C.c_int32), ("cols", C.c_void_p), ("S_out", C.c_void_p), ("S_final", C.c_void_p),
        ("h_cap", C.c_int64), ("h_rec", C.c_void_p), ("h_replay", C.c_void_p),
        ("n_replay", C.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(LIB_PATH)
        _lib.gso_solve.argtypes = [C.POINTER(_Problem)]
        _lib.gso_solve.restype = C.c_int
        _lib.gso_tableau.argtypes = [C.c_int, C.c_void_p, C.c_void_p]
        _lib.gso_rhs.argtypes = [C.c_int, C.c_double, C.c_void_p, C.c_void_p, C.c_int32,
                                 C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.gso_stiff_solve.argtypes = [C.POINTER(_Problem)]
        _lib.gso_stiff_solve.restype = C.c_int
        _lib.gso_stiff_rhs.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.gso_stiff_rhs.restype = C.c_int
        _lib.gso_rodas4.argtypes = [C.c_void_p]
        _lib.gso_rodas4.restype = C.c_int
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _strided(x, n, name):
    x = _f64(x)
    if x.ndim == 0 or x.size == 1:
        return x.reshape(1), 0
    if x.shape != (n,):
        raise ValueError(f"{name} must be a scalar or have shape ({n},)")
    return x, 1


def solve(rhs, tableau, y0, theta, t0, t1, rtol, atol, t_out=None, *, max_steps=10**7,
          h0=0.0, safety=0.9, alpha_min=0.2, alpha_max=5.0, beta1=0.0, beta2=0.0,
          no_grow_after_reject=False, nthreads=None, sens_cols=None, h_cap=0,
          h_replay=None, n_replay=None):
    """Solve an ensemble.

    y0: [d][n]; theta: [p] (shared) or [p][n]; t0, t1, rtol, atol: scalars or
    [n]; t_out: None, [K] (shared) or [K][n].  ``sens_cols`` lists columns of
    the forward sensitivity S = dy/dz, z = (y0 components, then parameters).
    Returns a dict of numpy arrays in the same SoA layouts.
    """
    rhs_id = RHS[rhs] if isinstance(rhs, str) else int(rhs)
    tab_id = TABLEAU[tableau] if isinstance(tableau, str) else int(tableau)
    d, p = DIM[rhs_id], NPARAM[rhs_id]
    y0 = _f64(y0)
    if y0.ndim != 2 or y0.shape[0] != d:
        raise ValueError(f"y0 must be [{d}][n]")
    n = y0.shape[1]
    theta = _f64(theta)
    if theta.ndim == 1:
        if theta.shape != (p,):
            raise ValueError("theta")
        th_stride = 0
    else:
        if theta.shape != (p, n):
            raise ValueError("theta")
        th_stride = n
    t0a, ts0 = _strided(t0, n, "t0")
    t1a, ts1 = _strided(t1, n, "t1")
    if ts0 != ts1:
        t0a = np.broadcast_to(t0a, (n,)).copy() if ts0 == 0 else t0a
        t1a = np.broadcast_to(t1a, (n,)).copy() if ts1 == 0 else t1a
        ts0 = 1
    rta, rs = _strided(rtol, n, "rtol")
    ata, as_ = _strided(atol, n, "atol")
    if rs != as_:
        rta = np.broadcast_to(rta, (n,)).copy() if rs == 0 else rta
        ata = np.broadcast_to(ata, (n,)).copy() if as_ == 0 else ata
        rs = 1
    if t_out is None:
        K, tk, tks = 0, None, 0
    else:
        tk = _f64(t_out)
        K = tk.shape[0]
        tks = 0 if tk.ndim == 1 else n
    out = {
        "y_final": np.zeros((d, n)),
        "n_accepted": np.zeros(n, np.int32),
        "n_rejected": np.zeros(n, np.int32),
        "status": np.zeros(n, np.int32),
    }
    y_out = np.zeros((d, K, n)) if K else None
    m = 0 if sens_cols is None else len(sens_cols)
    cols = np.ascontiguousarray(np.asarray(sens_cols if m else [0], np.int32))
    S_out = np.zeros((d, m, K, n)) if (m and K) else None
    S_final = np.zeros((d, m, n)) if m else None
    h_rec = None
    hr = nr = None
    if h_replay is not None:
        hr = _f64(h_replay)
        h_cap = hr.shape[1]
        nr = np.ascontiguousarray(np.asarray(n_replay, np.int32))
    elif h_cap:
        h_rec = np.zeros((n, h_cap))
    P = _Problem()
    P.rhs, P.tableau, P.n = rhs_id, tab_id, n
    P.y0, P.theta, P.theta_stride = _ptr(y0), _ptr(theta), th_stride
    P.t0, P.t1, P.t_stride = _ptr(t0a), _ptr(t1a), ts0
    P.rtol, P.atol, P.tol_stride = _ptr(rta), _ptr(ata), rs
    P.K, P.t_out, P.t_out_stride = K, _ptr(tk), tks
    P.y_out, P.y_final = _ptr(y_out), _ptr(out["y_final"])
    P.n_acc, P.n_rej, P.status = (_ptr(out["n_accepted"]), _ptr(out["n_rejected"]),
                                  _ptr(out["status"]))
    P.max_steps, P.h0 = int(max_steps), float(h0)
    P.safety, P.alpha_min, P.alpha_max = safety, alpha_min, alpha_max
    P.beta1, P.beta2 = beta1, beta2
    P.no_grow_after_reject = 1 if no_grow_after_reject else 0
    P.nthreads = nthreads or min(os.cpu_count() or 1, 16)
    P.m, P.cols, P.S_out, P.S_final = m, _ptr(cols), _ptr(S_out), _ptr(S_final)
    P.h_cap, P.h_rec, P.h_replay, P.n_replay = int(h_cap), _ptr(h_rec), _ptr(hr), _ptr(nr)
    stiff = rhs_id in STIFF_RHS or tab_id == TABLEAU["rodas4"]
    rc = (lib().gso_stiff_solve if stiff else lib().gso_solve)(C.byref(P))
    if rc != 0:
        raise ValueError(f"gso_solve rejected the problem (code {rc})")
    if K:
        out["y_out"] = y_out
    if m:
        out["S_final"] = S_final
        if K:
            out["S_out"] = S_out
    if h_rec is not None:
        out["h_rec"] = h_rec
    return out


def tableau(name):
    """Return the oracle's tableau as a dict of numpy arrays."""
    tid = TABLEAU[name] if isinstance(name, str) else int(name)
    ints = np.zeros(5, np.int32)
    dbl = np.zeros(10 + 100 + 10 + 10 + 80)
    lib().gso_tableau(tid, ints.ctypes.data, dbl.ctypes.data)
    s = int(ints[0])
    o = 0
    c = dbl[o:o + s]; o += s
    a = dbl[o:o + s * s].reshape(s, s); o += s * s
    b = dbl[o:o + s]; o += s
    bd = dbl[o:o + s]; o += s
    P = dbl[o:o + s * 8].reshape(s, 8)
    return {"s": s, "order": int(ints[1]), "fsal": bool(ints[2]), "dense": int(ints[3]),
            "deg": int(ints[4]), "c": c.copy(), "a": a.copy(), "b": b.copy(),
            "bdiff": bd.copy(), "P": P[:, :int(ints[4])].copy()}


def rhs(name, t, y, theta, sens_cols=None):
    """f(t, y, theta) at one point, and optionally Jacobian columns [d][m]."""
    rid = RHS[name] if isinstance(name, str) else int(name)
    d = DIM[rid]
    y = _f64(y)
    theta = _f64(theta)
    f = np.zeros(d)
    m = 0 if sens_cols is None else len(sens_cols)
    cols = np.ascontiguousarray(np.asarray(sens_cols if m else [0], np.int32))
    J = np.zeros((d, max(m, 1)))
    rc = lib().gso_rhs(rid, float(t), y.ctypes.data, theta.ctypes.data, m, cols.ctypes.data,
                       f.ctypes.data, J.ctypes.data)
    if rc != 0:
        raise ValueError("gso_rhs")
    return (f, J[:, :m]) if m else f


def stiff_rhs(name, y, theta):
    """f and the analytic Jacobian [d][d] of a stiff kinetics right-hand side."""
    rid = RHS[name] if isinstance(name, str) else int(name)
    d = DIM[rid]
    y, theta = _f64(y), _f64(theta)
    f = np.zeros(d)
    J = np.zeros((d, d))
    if lib().gso_stiff_rhs(rid, y.ctypes.data, theta.ctypes.data, f.ctypes.data,
                           J.ctypes.data) != 0:
        raise ValueError("gso_stiff_rhs")
    return f, J


def rodas4():
    """Standard-form Rodas4 coefficients derived by the oracle: gamma, alpha,
    Gamma (lower triangular, diagonal gamma), b, bhat."""
    out = np.zeros(1 + 36 + 36 + 12)
    lib().gso_rodas4(out.ctypes.data)
    return {"gamma": out[0], "alpha": out[1:37].reshape(6, 6), "Gamma": out[37:73].reshape(6, 6),
            "b": out[73:79], "bhat": out[79:85]}
