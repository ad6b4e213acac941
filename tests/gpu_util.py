"""Helpers shared by the GPU tests: run a workload dict through the HIP path
and through the oracle on the same seeded inputs."""
import numpy as np
import torch

from paper_2609_28458_amd import api


def gpu_solve(w, launch=None, n=None, order=None, **kw):
    sl = slice(None) if n is None else slice(0, n)
    y0 = w["y0"][:, sl]
    th = w["theta"] if np.ndim(w["theta"]) == 1 else w["theta"][:, sl]

    def cut(x):
        return x[sl] if np.ndim(x) == 1 and np.size(x) == w["y0"].shape[1] else x

    to = w.get("t_out")
    if to is not None and np.ndim(to) == 2:
        to = to[:, sl]
    prob = api.make_problem(w["rhs"], kw.get("tableau", w["tableau"]), y0, th, cut(w["t0"]),
                            cut(w["t1"]), cut(w["rtol"]), cut(w["atol"]), to)
    sol = api.solve(prob, launch or api.Launch(), order=order)
    torch.cuda.synchronize()
    return sol


def to_np(sol):
    out = {"y_final": sol.y_final.cpu().numpy(), "n_accepted": sol.n_accepted.cpu().numpy(),
           "n_rejected": sol.n_rejected.cpu().numpy(), "status": sol.status.cpu().numpy()}
    if sol.y_out is not None:
        out["y_out"] = sol.y_out.cpu().numpy()
    return out


def oracle_solve(orc, w, idx=None, **kw):
    idx = np.arange(w["y0"].shape[1]) if idx is None else np.asarray(idx)
    n_all = w["y0"].shape[1]

    def cut(x):
        return np.asarray(x)[idx] if np.ndim(x) == 1 and np.size(x) == n_all else x

    th = w["theta"] if np.ndim(w["theta"]) == 1 else w["theta"][:, idx]
    to = w.get("t_out")
    if to is not None and np.ndim(to) == 2:
        to = to[:, idx]
    return orc.solve(w["rhs"], kw.pop("tableau", w["tableau"]), w["y0"][:, idx], th,
                     cut(w["t0"]), cut(w["t1"]), cut(w["rtol"]), cut(w["atol"]), to, **kw)


def rel_err(a, b):
    """|a - b| / max(|b|, 1), elementwise (state components are O(1))."""
    return np.abs(a - b) / np.maximum(np.abs(b), 1.0)
