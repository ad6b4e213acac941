"""The algorithmic flop counts the benchmark divides by (bench.py,
FLOPS_PER_ATTEMPT / FLOPS_PER_NODE) against the same formula evaluated on the
oracle's own tableaux: stage sums 2 d (nnz(A) + s - 1), the update of a
non-FSAL pair 2 d (nnz(b) + 1), stage times 2 (s - 1), error weights
2 d nnz(b - bhat) + d, norm 5 d + 2, controller 5, and F_f per new stage.
F_f is the hand count of each right-hand side as the kernels evaluate it
(13 for the log halo, 119 for precession)."""
import numpy as np

import bench

F_F = {"loghalo": 13, "spinprec": 119}
DIM = {"loghalo": 6, "spinprec": 9}


def _parts(orc, tab, rhs):
    t = orc.tableau(tab)
    s, d = t["s"], DIM[rhs]
    nnz_a = int(np.count_nonzero(t["a"]))
    nnz_b = int(np.count_nonzero(t["b"]))
    nnz_e = int(np.count_nonzero(t["bdiff"]))
    update = 0 if t["fsal"] else 2 * d * (nnz_b + 1)
    s_new = s - 1 if t["fsal"] else s
    attempt = (2 * d * (nnz_a + s - 1) + update + 2 * (s - 1) + 2 * d * nnz_e + d
               + 5 * d + 2 + 5 + s_new * F_F[rhs])
    node = (s - 1) * F_F[rhs] + 2 * d * (nnz_a + s - 1) + update
    return attempt, node


def test_flops_per_attempt_follow_the_tableaux(orc):
    for (tab, rhs), flops in bench.FLOPS_PER_ATTEMPT.items():
        assert _parts(orc, tab, rhs)[0] == flops, (tab, rhs)
    for (tab, rhs), flops in bench.FLOPS_PER_NODE.items():
        assert _parts(orc, tab, rhs)[1] == flops, (tab, rhs)


def test_stiff_flops_formula():
    assert bench.rodas4_flops_per_attempt(8, 6, 28) == 1918
    assert bench.rodas4_flops_per_attempt(3, 3, 7) == 419
