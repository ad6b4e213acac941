"""The algorithmic flop counts the benchmark divides by (bench.py,
FLOPS_PER_ATTEMPT / FLOPS_PER_NODE) against the same formula evaluated on the
oracle's own tableaux: stage sums 2 d (nnz(A) + s - 1), the update of a
non-FSAL pair 2 d (nnz(b) + 1), stage times 2 (s - 1), error weights
2 d nnz(b - bhat) + d, norm 5 d + 2, controller 5, and F_f per new stage;
per output node a polynomial evaluation or a shortened step.
F_f is the hand count of each right-hand side in its unfolded form, with
products of parameters alone taken once per trajectory: 13 for the log halo;
119 for precession, the form the adjoint differentiates (SpinPrec::forward and
the products that turn it into dy).  The precession solve evaluates a folded
form of the same function with 97 (the reciprocal of dv/dt folded into the
precession coefficients, eta into the prepared coefficients), so its achieved
rate counts the unfolded work."""
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
    if t["deg"] > 0:
        # polynomial output: the weights b_j(sigma) by Horner (2 deg + 2 each),
        # d sums of s terms and the final fma, and sigma itself
        node = s * (2 * t["deg"] + 2) + d * (2 * s + 2) + 2
    else:
        # a shortened step from the start of the step
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


V_F = {"loghalo": 46}  # the log halo's VJP as the kernels evaluate it


def test_flops_per_vjp_step_follow_the_tableau(orc):
    """Reverse of one accepted step: the first right-hand side; for every
    stage j >= 1 that feeds the step (b_j != 0 or a later a_ij != 0) its
    stage sum 2 d (nnz(row j) + 1), stage time 2 and, unless it is the last
    stage, its right-hand side; the seeds h b_j lam (1 + d per nonzero b_j);
    then for every feeding stage the VJP, the d-term accumulation into y,
    the stage time for j >= 1, and (1 + 2 d) per nonzero a_jl of its row."""
    for (tab, rhs), flops in bench.FLOPS_PER_VJP_STEP.items():
        t = orc.tableau(tab)
        s, d, a, b = t["s"], DIM[rhs], np.asarray(t["a"]), np.asarray(t["b"])
        feeds = [b[j] != 0 or np.any(a[j + 1:, j] != 0) for j in range(s)]
        nnz_row = [int(np.count_nonzero(a[j, :j])) for j in range(s)]
        total = F_F[rhs]
        for j in range(1, s):
            if feeds[j]:
                total += 2 * d * (nnz_row[j] + 1) + 2 + (F_F[rhs] if j < s - 1 else 0)
        total += int(np.count_nonzero(b)) * (1 + d)
        for j in range(s):
            if feeds[j]:
                total += V_F[rhs] + d + (2 if j >= 1 else 0) + nnz_row[j] * (1 + 2 * d)
        assert total == flops, (tab, rhs, total)
