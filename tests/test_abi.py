"""The C-ABI library loads, exports every symbol include/gradsolve.h declares,
and rejects bad arguments on the host before touching the GPU (these calls
run without a GPU)."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2609_28458_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "gradsolve.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(gs_[a-z_]+)\s*\(", src)
    return sorted(set(names))


def test_header_symbols_exported():
    names = declared_functions()
    assert "gs_solve" in names and "gs_solve_vjp" in names and "gs_dense_eval" in names
    lib = C.CDLL(api.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(api.EXPORTS) == set(names)


MIRRORED = {"gs_controller": api.gs_controller, "gs_solve_args": api.gs_solve_args,
            "gs_vjp_args": api.gs_vjp_args, "gs_sens_args": api.gs_sens_args,
            "gs_de_profile_args": api.gs_de_profile_args}


def _c_layout(tmp_path):
    """sizeof and offsetof of every field of every mirrored struct, printed by
    a C program compiled against include/gradsolve.h."""
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gradsolve.h"',
             "int main(void) {"]
    for name, cls in MIRRORED.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            cname = "lambda" if fname == "lambda_" else fname
            lines.append(f'  printf("{name} {fname} %zu\\n", offsetof({name}, {cname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-I",
                           os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)], text=True)
    return {tuple(line.split()[:2]): int(line.split()[2]) for line in out.splitlines()}


def test_every_mirrored_struct_matches_the_c_layout(tmp_path):
    """Every struct the binding mirrors has the C header's size and field
    offsets (a field the header lacks, or one out of place, fails here)."""
    c = _c_layout(tmp_path)
    for name, cls in MIRRORED.items():
        assert C.sizeof(cls) == c[(name, "size")], name
        for fname, _ in cls._fields_:
            assert getattr(cls, fname).offset == c[(name, fname)], (name, fname)


def test_struct_layout_matches_header():
    # offsets the binding relies on: compare the ctypes size with the C size
    # reported through the default-args call (the library zero-fills exactly
    # sizeof(gs_solve_args) bytes, so a larger ctypes struct keeps a sentinel).
    buf = (C.c_ubyte * (C.sizeof(api.gs_solve_args) + 64))()
    for i in range(len(buf)):
        buf[i] = 0xAB
    api.lib().gs_default_args(C.cast(buf, C.POINTER(api.gs_solve_args)))
    assert buf[C.sizeof(api.gs_solve_args)] == 0xAB
    assert all(buf[i] != 0xAB or i >= C.sizeof(api.gs_solve_args) for i in range(len(buf)))
    a = api.gs_default_args()
    assert a.ctrl.safety == 0.9 and a.ctrl.alpha_min == 0.2 and a.ctrl.alpha_max == 5.0
    assert a.max_steps == 10_000_000


def _args(**kw):
    a = api.gs_default_args()
    a.rhs, a.tableau, a.n, a.d, a.p = 2, 0, 1000, 6, 3
    for f in ("y0", "theta", "t0", "t1", "rtol", "atol", "y_final", "n_accepted",
              "n_rejected", "status"):
        setattr(a, f, 0x1000)
    a.workspace = 0x100000
    a.workspace_bytes = 1 << 30
    for k, v in kw.items():
        setattr(a, k, v)
    return a


@pytest.mark.parametrize("kw", [
    dict(rhs=9), dict(tableau=4), dict(d=5), dict(p=4), dict(n=-1),
    dict(y0=None), dict(theta_stride=5), dict(t_stride=2), dict(K=3),
    dict(ckpt_every=-1), dict(ckpt_every=4, ckpt_capacity=0), dict(block=100), dict(wide=-1),
    dict(block=1024), dict(refill=65), dict(schedule=5),
])
def test_invalid_arguments_rejected(kw):
    assert api.lib().gs_solve(C.byref(_args(**kw))) == 1


def test_workspace_checks():
    a = _args(workspace=None)
    assert api.lib().gs_solve(C.byref(a)) == 3
    a = _args(ckpt_every=8, ckpt_capacity=100)
    need = api.gs_workspace_bytes(a)
    # counters + tape (n * cap * (3 + 2d) doubles) + replay scratch (lanes * k * (2 + d))
    # + running cotangents (lanes * (d + p), one loss per launch), every part a
    # multiple of 256 bytes, then the n 32-bit tape slots
    assert need == 256 + 1000 * 100 * 15 * 8 + 1024 * 8 * 8 * 8 + 1024 * 9 * 8 + 1000 * 4
    store = api.gs_workspace_bytes(_args(ckpt_every=1, ckpt_capacity=100))
    # store mode: records of 2 + d doubles and no replay scratch
    assert store == 256 + 1000 * 100 * 8 * 8 + 1024 * 9 * 8 + 1000 * 4
    a.workspace_bytes = need - 1
    assert api.lib().gs_solve(C.byref(a)) == 3
    a = _args(workspace=0x100010)
    assert api.lib().gs_solve(C.byref(a)) == 3


def test_vjp_requires_tape():
    a = _args()
    v = api.gs_vjp_args(1, None, 0x1000, 0x1000, 0x1000, 0, 0, None)
    assert api.lib().gs_solve_vjp(C.byref(a), C.byref(v)) == 5



def test_vjp_groups_need_a_store_tape_and_final_state_losses():
    v = api.gs_vjp_args(1, None, 0x1000, 0x1000, 0x1000, 0, 0, None, -1)
    store = dict(ckpt_every=1, ckpt_capacity=10)
    assert api.lib().gs_solve_vjp(C.byref(_args(**store)), C.byref(v)) == 1
    v.wide = 8
    assert api.lib().gs_solve_vjp(C.byref(_args(ckpt_every=4, ckpt_capacity=10)), C.byref(v)) == 2
    nodes = dict(K=3, t_out=0x1000, y_out=0x1000)
    assert api.lib().gs_solve_vjp(C.byref(_args(**store, **nodes)), C.byref(v)) == 2

def test_status_strings():
    for code in range(6):
        assert api.lib().gs_status_string(code)
    assert api.gs_version() == "0.2.0"


def test_wide_needs_the_queue_schedule():
    # groups of lanes take the queue schedule
    assert api.lib().gs_solve(C.byref(_args(wide=8, schedule=1))) == 2
    # output nodes and both tape modes pass the host checks (the call then fails
    # only for want of a GPU)
    for kw in (dict(wide=8, K=3, t_out=0x1000, y_out=0x1000),
               dict(wide=8, ckpt_every=4, ckpt_capacity=10)):
        assert api.lib().gs_solve(C.byref(_args(**kw))) != 2


def test_sens_argument_checks():
    a = _args()
    cols = (C.c_int32 * 2)(0, 8)
    ok = api.gs_sens_args(2, C.cast(cols, C.c_void_p), 0x1000, 0)
    assert api.lib().gs_solve_sens(C.byref(_args()), None) == 1
    assert api.lib().gs_solve_sens(C.byref(a), C.byref(api.gs_sens_args(0, C.cast(cols, C.c_void_p), 0x1000, 0))) == 1
    bad = (C.c_int32 * 2)(0, 9)  # d + p = 9 columns exist
    assert api.lib().gs_solve_sens(C.byref(a), C.byref(api.gs_sens_args(2, C.cast(bad, C.c_void_p), 0x1000, 0))) == 1
    # no tape with sensitivities; wide groups need the queue schedule
    assert api.lib().gs_solve_sens(C.byref(_args(ckpt_every=4, ckpt_capacity=10)), C.byref(ok)) == 2
    assert api.lib().gs_solve_sens(C.byref(_args(wide=8, schedule=1)), C.byref(ok)) == 2


def _de_args(**kw):
    a = api.gs_de_profile_args()
    a.n, a.K, a.K_data = 1000, 64, 7
    for f in ("lambda_", "omega_m", "h", "a0", "N_nodes", "N_data", "data", "sigma", "chi2",
              "chi2_prev", "decrement", "status"):
        setattr(a, f, 0x1000)
    a.iters, a.newton, a.mu, a.trust_om, a.trust_h = 20, 3, 1e-3, 0.05, 0.05
    a.tableau, a.N_start, a.rtol, a.atol = 0, -3.9, 1.78e-4, 1.78e-7
    a.workspace = 0x100000
    for k, v in kw.items():
        setattr(a, k, v)
    return a


def _al(x):
    return (x + 255) // 256 * 256


def test_de_profile_workspace_and_argument_checks():
    L = api.lib()
    n, K, Kd = 1000, 64, 7
    direct = sum(_al(b) for b in (256, 32, 4 * n * 8, 3 * n * 8, 3 * K * n * 8, 3 * n * 8,
                                  6 * K * n * 8, 6 * n * 8, 4 * n, 4 * n, 4 * n, 0, 0, 0))
    spline = direct + _al(Kd * K * 8) + _al(3 * K * K * 8)
    assert L.gs_de_profile_workspace_bytes(C.byref(_de_args(K_data=0))) == direct
    assert L.gs_de_profile_workspace_bytes(C.byref(_de_args())) == spline
    assert L.gs_de_profile_workspace_bytes(C.byref(_de_args(K_data=-1))) == 0
    assert L.gs_de_profile(C.byref(_de_args(workspace_bytes=spline - 1))) == 3
    assert L.gs_de_profile(C.byref(_de_args(workspace=0x100001, workspace_bytes=spline))) == 3
    for bad in (dict(K_data=-1), dict(K=3), dict(N_data=None), dict(iters=-1), dict(newton=-1),
                dict(N_start=0.0), dict(trust_h=0.0), dict(tableau=3), dict(data=None)):
        assert L.gs_de_profile(C.byref(_de_args(workspace_bytes=spline, **bad))) == 1, bad
    # n = 0 is a no-op, whatever the pointers
    assert L.gs_de_profile(C.byref(_de_args(n=0, workspace=None))) == 0


def _stiff(**kw):
    a = _args(rhs=5, tableau=3, d=3, p=3)
    for k, v in kw.items():
        setattr(a, k, v)
    return a


def test_stiff_path_argument_checks():
    L = api.lib()
    # explicit pair on a stiff right-hand side, Rodas4 on an explicit one
    assert L.gs_solve(C.byref(_args(rhs=5, tableau=0, d=3, p=3))) == 2
    assert L.gs_solve(C.byref(_args(tableau=3))) == 2
    assert L.gs_solve(C.byref(_stiff(d=8))) == 1
    assert L.gs_solve(C.byref(_stiff(rhs=6, d=8, p=11))) == 1
    # no tape, no wide groups, the default output layout, I control only
    assert L.gs_solve(C.byref(_stiff(ckpt_every=1, ckpt_capacity=10))) == 2
    assert L.gs_solve(C.byref(_stiff(wide=4))) == 2
    assert L.gs_solve(C.byref(_stiff(out_layout=1))) == 2
    b = _stiff()
    b.ctrl.beta2 = 0.04
    assert L.gs_solve(C.byref(b)) == 2
    # workspace: the queue counters only
    assert L.gs_workspace_bytes(C.byref(_stiff(rhs=6, d=8, p=12))) == 256
    # entry points the stiff path does not have
    v = api.gs_vjp_args(1, None, 0x1000, 0x1000, 0x1000, 0, 0, None)
    assert L.gs_solve_vjp(C.byref(_stiff()), C.byref(v)) == 2
    cols = (C.c_int32 * 1)(0)
    s = api.gs_sens_args(1, C.cast(cols, C.c_void_p), 0x1000, 0)
    assert L.gs_solve_sens(C.byref(_stiff()), C.byref(s)) == 2
    assert L.gs_dense_eval(C.byref(_stiff()), 1, 0x1000, 0x1000, None) == 2
    assert L.gs_rhs_eval(5, 10, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000,
                         None) == 2
    assert L.gs_rhs_eval(9, 10, 0x1000, 0x1000, 0x1000, 0x1000, None, None, None, None) == 1


def test_size_limits():
    L = api.lib()
    assert L.gs_de_profile(C.byref(_de_args(n=(1 << 31) + 1, workspace_bytes=1 << 40))) == 2
    assert L.gs_rhs_eval(2, (1 << 31) + 1, 0x1000, 0x1000, 0x1000, 0x1000, None, None, None,
                         None) == 2
    assert L.gs_solve(C.byref(_args(n=(1 << 31) + 1))) == 2


def test_output_layout_argument():
    """out_layout is 0 ([d][K][n]) or 1 ([K][n][d]); anything else is rejected
    before a launch."""
    L = api.lib()
    for bad in (-1, 2, 7):
        assert L.gs_solve(C.byref(_args(out_layout=bad))) == 1
    assert api.OUT_LAYOUT == {"dkn": 0, "knd": 1}


def test_queue_order_argument_checks():
    a = _args()
    ws = (C.c_ubyte * 512)()
    lib = api.lib()
    # no order buffer
    assert lib.gs_queue_order(C.byref(a), None, None, C.addressof(ws), 512) == 1
    # workspace smaller than gs_queue_order_workspace_bytes(n)
    need = lib.gs_queue_order_workspace_bytes(a.n)
    assert need >= 12 * a.n + 65536 * 4
    assert lib.gs_queue_order(C.byref(a), None, 0x1000, 0x100000, need - 1) == 3
    # misaligned workspace
    assert lib.gs_queue_order(C.byref(a), None, 0x1000, 0x100008, need) == 3
    # the built-in model needs the spans and tolerances
    assert lib.gs_queue_order(C.byref(_args(t1=None)), None, 0x1000, 0x100000, need) == 1
    assert lib.gs_queue_order_workspace_bytes(-1) == 0
    # n = 0: nothing to do
    assert lib.gs_queue_order(C.byref(_args(n=0)), None, None, None, 0) in (0, 1)


def test_noalloc_argument_checks():
    """The allocation-free solve rejects a tape before touching the device."""
    lib = api.lib()
    assert lib.gs_solve_noalloc(C.byref(_args(ckpt_every=1, ckpt_capacity=10))) == 2
    assert lib.gs_solve_noalloc(None) == 1
    assert lib.gs_status_string(6) == b"request exceeds the fixed static scratch of gs_solve_noalloc"
