/*
 * gradsolve -- ensemble solve and discrete-adjoint gradients of many small
 * independent ODE systems on one AMD Instinct MI355X (gfx950).
 *
 * The problem is the paper's ensemble initial-value problem (Section "The
 * ensemble problem", eq:ivp): n independent systems dy_i/dt = f(t, y_i,
 * theta_i), y_i(t0_i) = y0_i, each read at output times t_k.  Every
 * trajectory is integrated by an explicit Runge--Kutta pair with its own
 * adaptive step (Appendix "Runge--Kutta steps and error control": eq:rk,
 * eq:errnorm, eq:controller), outputs inside a step come from the dense
 * polynomial or, for Verner 7, a shortened step (eq:dense), and gradients of
 * scalar losses are the exact derivative of the discrete solution with the
 * accepted steps held fixed (Appendix "Derivatives", eq:stage-sens; here
 * computed in reverse mode, the transpose of that recursion).
 *
 * Conventions shared by every entry point:
 *  - All array pointers are DEVICE pointers owned by the caller.  The
 *    library never allocates or frees memory in these calls, so they can be
 *    captured in a HIP graph.  Arrays are float64 or int32 as declared.
 *  - Layouts are structure-of-arrays with the trajectory index fastest:
 *    a state is [d][n], outputs are [d][K][n].
 *  - A "stride" of 0 broadcasts one value (or vector) to all trajectories.
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream).  Argument errors are detected on the host before anything is
 *    launched and returned as a gs_status; nothing is launched then.
 *  - Numerical failures of single trajectories are NOT call errors: the
 *    call returns GS_OK and status[i] carries a gs_traj_status.
 *  - Nothing throws across this boundary.
 */
#ifndef GRADSOLVE_H
#define GRADSOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gs_status {
  GS_OK = 0,
  GS_ERR_INVALID = 1,     /* bad argument (null pointer, size, layout, order) */
  GS_ERR_UNSUPPORTED = 2, /* valid request the library does not implement    */
  GS_ERR_WORKSPACE = 3,   /* workspace missing or smaller than required      */
  GS_ERR_HIP = 4,         /* a HIP runtime call failed                       */
  GS_ERR_NO_TAPE = 5,     /* gradient requested but the solve kept no tape   */
  GS_ERR_TOO_LARGE = 6    /* the request needs more scratch than the fixed
                             static buffer of gs_solve_noalloc holds         */
} gs_status;

/* Per-trajectory outcome written to status[i]. */
typedef enum gs_traj_status {
  GS_TRAJ_OK = 0,
  GS_TRAJ_MAX_STEPS = 1,     /* max_steps attempts without reaching t1        */
  GS_TRAJ_DT_UNDERFLOW = 2,  /* |h| < 16 eps max(|t|, 1)                      */
  GS_TRAJ_NONFINITE = 3,     /* non-finite y0 or state, or 50 NaN rejections  */
  GS_TRAJ_TAPE_OVERFLOW = 4, /* reached t1, but more checkpoints than the
                                capacity: the trajectory cannot be replayed   */
  GS_TRAJ_BAD_INPUT = 5,     /* t1 < t0, rtol <= 0, atol < 0, or output nodes
                                not non-decreasing within [t0, t1]; checked
                                on the device, nothing integrated, outputs NaN */
  GS_TRAJ_NOT_RUN = 6        /* a queue order was given and this index never
                                appeared in it (the order was not a
                                permutation): nothing was written for it     */
} gs_traj_status;

/* Runge--Kutta pairs (Section "Adaptive integration"). */
typedef enum gs_tableau_id {
  GS_DOPRI5 = 0,  /* Dormand & Prince 5(4), FSAL, 4th-order continuous output */
  GS_TSIT5 = 1,   /* Tsitouras 5(4), FSAL, 4th-order interpolant              */
  GS_VERNER7 = 2, /* Verner 7(6), 10 stages, outputs by shortened steps       */
  GS_RODAS4 = 3   /* stiff path: Rosenbrock method Rodas4 (Hairer & Wanner;
                     order 4, embedded 3, stiffly accurate) with the
                     analytic Jacobian, for the stiff right-hand sides only;
                     outputs are landed on (the step is shortened to end at
                     each output time) instead of interpolated             */
} gs_tableau_id;

/* Right-hand sides; each fixes d (state size) and p (parameter count). */
typedef enum gs_rhs_id {
  GS_RHS_HARMONIC = 0, /* d=2 (x, v), p=1 (omega)                           */
  GS_RHS_KEPLER = 1,   /* d=4 (x, y, vx, vy), p=1 (mu)                      */
  GS_RHS_LOGHALO = 2,  /* d=6 (x, v), p=3 (v0, q, rc); eq:loghalo           */
  GS_RHS_SPINPREC = 3, /* d=9 (L, S1, S2 unit vectors) in v, p=3 (q, chi1,
                          chi2); eq:prec-spins, eq:prec-L, eq:prec-omega,
                          eq:prec-rr with 2PN radiation reaction              */
  GS_RHS_QUINT = 4,    /* d=3 (phi, u, I) in N = ln a, p=4 (a0, lambda,
                          Omega_m, Omega_r); eq:de-model, eq:de-rhs          */
  /* Stiff mass-action kinetics, autonomous, GS_RODAS4 only: */
  GS_RHS_KIN3 = 5,     /* d=3 (a, b, c), p=3 (k1, k2, k3): a -> b (k1 a),
                          b + c -> 2c (k2 b c), c -> a (k3 c)               */
  GS_RHS_KIN8 = 6,     /* d=8, p=12 (k1..k10, s, k12): y1 <-> y2 (k1, k2),
                          y2 -> y3 (k3), y3 <-> y4 (k4, k5), y4 + y5 <-> y6
                          (k6 y4 y5, k7 y6), y6 -> y7 (k8), y7 -> y8 (k9),
                          y8 -> y1 (k10), source s -> y5, y5 -> sink (k12) */
  /* The classic stiff chemistry problems named with the paper's Rosenbrock
     kernel (Discussion), standard form, rate constants as parameters: */
  GS_RHS_ROBER = 7,    /* Robertson (1966), d=3, p=3 (k1, k2, k3), nominal
                          (0.04, 3e7, 1e4): y1' = -k1 y1 + k3 y2 y3,
                          y2' = k1 y1 - k3 y2 y3 - k2 y2^2, y3' = k2 y2^2    */
  GS_RHS_HIRES = 8     /* HIRES (Schaefer 1975), d=8, p=8 (a, b, c, s, d, e,
                          kf, g), nominal (1.71, 0.43, 8.32, 0.0007, 0.035,
                          1.12, 280, 0.69); the problem's constants 8.75,
                          10.03, 1.745, 1.81 are c+b, c+a, a+d, e+g         */
} gs_rhs_id;

/* How trajectories are handed to lanes. */
typedef enum gs_schedule {
  GS_SCHED_QUEUE = 0, /* persistent grid; lanes retire and refill from an
                         atomic work queue                                   */
  GS_SCHED_STATIC = 1 /* one lane per trajectory, no refill (a lane waits for
                         the slowest lane of its wavefront)                  */
} gs_schedule;

/* Step-size controller, eq:controller generalised to PI form:
 *   h_new = h * min(alpha_max, max(alpha_min,
 *                    safety * err^(-beta1) * err_prev^(beta2)))
 * with err_prev the (floored at 1e-4) norm of the last accepted step.
 * beta1 <= 0 selects 1/nu; beta2 = 0 is the paper's I controller. */
typedef struct gs_controller {
  double safety;    /* paper: "< 1"; 0.9 by default                 */
  double alpha_min; /* paper: 0.2                                   */
  double alpha_max; /* paper: 5                                     */
  double beta1;
  double beta2;
} gs_controller;

/* One ensemble solve.  Sizes: d and p must equal those of `rhs`. */
typedef struct gs_solve_args {
  int32_t rhs;     /* gs_rhs_id                                             */
  int32_t tableau; /* gs_tableau_id                                         */
  int64_t n;       /* trajectories (0 allowed: nothing is launched)         */
  int32_t d, p;

  const double* y0;      /* [d][n]                                          */
  const double* theta;   /* [p][theta_stride] (stride 0: shared [p] vector)  */
  int64_t theta_stride;  /* 0 or n                                          */
  const double* t0;      /* [t_stride]; t1[i] >= t0[i]                      */
  const double* t1;
  int64_t t_stride;      /* 0 or 1                                          */
  const double* rtol;    /* [tol_stride], > 0                               */
  const double* atol;    /* [tol_stride], >= 0                              */
  int64_t tol_stride;    /* 0 or 1                                          */

  int32_t K;             /* output nodes per trajectory (0 = none)          */
  const double* t_out;   /* [K][t_out_stride], non-decreasing in k, each in
                            [t0, t1] of its trajectory                      */
  int64_t t_out_stride;  /* 0 or n                                          */

  double* y_out;         /* [d][K][n], or NULL when K == 0                  */
  double* y_final;       /* [d][n]                                          */
  int32_t* n_accepted;   /* [n]                                             */
  int32_t* n_rejected;   /* [n]                                             */
  int32_t* status;       /* [n] gs_traj_status                              */

  int64_t max_steps;     /* attempts per trajectory; <= 0: 10^7             */
  double h0;             /* > 0: first step; <= 0: Hairer-Norsett-Wanner
                            starting-step rule                              */
  gs_controller ctrl;

  /* Gradient tape (the store-or-recompute choice of eq:cost), up to
     ckpt_capacity records per trajectory:
       ckpt_every = 0   no tape (no gradient; dense queries replay from t0);
       ckpt_every = 1   store mode: (t_n, h_{n-1}, y_n) of every accepted
                        step, n = 0..N, so capacity >= N + 1; the adjoint
                        and dense queries replay nothing;
       ckpt_every >= 2  checkpoint mode: (t, h, err_prev, y, f(t, y)) every
                        ckpt_every accepted steps; the adjoint replays each
                        segment, so capacity >= N / ckpt_every + 1.
     A trajectory that needs more records ends with GS_TRAJ_TAPE_OVERFLOW
     (its solution is still complete). */
  int32_t ckpt_every;
  int32_t ckpt_capacity;

  /* Launch shape (0 = choose automatically). */
  int32_t schedule;      /* gs_schedule                                     */
  int32_t block;         /* lanes per workgroup: 64, 128, 192 or 256        */
  int32_t grid;          /* workgroups of the persistent grid               */
  int32_t refill;        /* refill a wavefront once this many lanes idle,
                            1..64 (0: 8)                                    */
  int32_t wide;          /* the first `wide` trajectories of the queue order
                            run on 16 lanes each (one state component per
                            lane) in the same launch, for the long tail of
                            uneven ensembles; results are bit-identical to
                            one lane per trajectory.  0 = none.  Needs the
                            queue schedule (else GS_ERR_UNSUPPORTED); the
                            tape (either mode) and output nodes are written
                            record for record as one lane writes them, and
                            gs_solve_sens carries its tangents on the same
                            groups (gs_solve_vjp has a `wide` of its own).
                            Explicit pairs only.  The groups
                            refill from their own queue; they and the single
                            lanes share the grid (the occupancy limit, or
                            `grid` when given), the single lanes keeping up
                            to half of it, each side at least one
                            workgroup.                                      */
  const int64_t* order;  /* [n] queue order (a permutation of 0..n-1), or
                            NULL for 0, 1, ..., n-1; gs_solve_vjp takes the
                            trajectories in the same order.  Device memory,
                            read on the device only: entries outside [0, n)
                            are skipped, and before the solve every status
                            is set to GS_TRAJ_NOT_RUN, so an index the order
                            misses keeps that status (and gs_solve_vjp gives
                            it NaN cotangents).  gs_queue_order builds a
                            longest-first order on the device.              */

  void* workspace;       /* device memory, >= gs_workspace_bytes(args),
                            256-byte aligned.  Bytes 16..23 hold a uint64
                            count of adjoint segment replays that did not
                            reproduce the next checkpoint bit-exactly
                            (diagnostic; reset by each gs_solve_vjp).      */
  size_t workspace_bytes;
  void* stream;          /* hipStream_t                                     */
  int32_t out_layout;    /* layout of y_out: 0 = [d][K][n] (the default);
                            1 = [K][n][d], the d components of one output of
                            one trajectory adjacent, so an output costs one
                            cache line in HBM instead of d.  Explicit
                            tableaux only (GS_RODAS4 with 1:
                            GS_ERR_UNSUPPORTED); any other value:
                            GS_ERR_INVALID.                                 */
} gs_solve_args;

/* Cotangents for gs_solve_vjp.  R independent scalar losses over the same
 * tape, one adjoint launch each: for each r, ybar_out[r] = dL_r/dy(t_k) and
 * ybar_final[r] = dL_r/dy(t1). */
typedef struct gs_vjp_args {
  int32_t R;                /* 1 <= R <= 8                                  */
  const double* ybar_out;   /* [R][d][K][n] or NULL                         */
  const double* ybar_final; /* [R][d][n] or NULL                            */
  double* y0bar;            /* [R][d][n]  out: dL_r/dy0                     */
  double* thetabar;         /* [R][p][n]  out: dL_r/dtheta_i per trajectory;
                               for shared theta the caller sums over n      */
  int32_t block;            /* 0 = automatic                                */
  int32_t grid;             /* 0 = automatic                                */
  void* stream;             /* hipStream_t                                  */
  int32_t wide;             /* the first `wide` positions of the queue order
                               reversed on 16 lanes each (one component per
                               lane), bitwise as one lane reverses them;
                               store-mode tapes (ckpt_every 1) of losses on
                               the final state only (K = 0), else
                               GS_ERR_UNSUPPORTED.  0 = none.  The groups and
                               the single lanes share the grid as for
                               gs_solve's `wide`.                           */
} gs_vjp_args;

/* Fill a gs_solve_args with defaults: the paper's controller (safety 0.9,
 * alpha 0.2 / 5, I control), automatic h0, max_steps 10^7, queue schedule,
 * automatic launch shape, no tape.  Pointers are zeroed. */
void gs_default_args(gs_solve_args* args);

/* Bytes of workspace `args` needs: the work-queue counters, the tape
 * (n * ckpt_capacity records of 2 + d doubles in store mode, 3 + 2d in
 * checkpoint mode; a trajectory's records sit in the slot of the queue
 * position it was taken from, and n 32-bit slot numbers follow at the end
 * of the workspace) and, with a tape, the adjoint's per-lane buffers for
 * min(n rounded up to 256, 131072) lanes: the running cotangents (d + p
 * doubles) and, in checkpoint mode, the replay scratch (ckpt_every steps of
 * 2 + d doubles); for an explicit pair with K > 0 also (2 + d) K n doubles
 * for the outputs inside steps (start time, length and start state of the
 * step that passes each), which gs_solve evaluates after the solve kernel
 * (one thread per output: the dense polynomial of the step taken again, or
 * Verner 7's shortened step).
 * Returns 0 for an invalid `args`. */
size_t gs_workspace_bytes(const gs_solve_args* args);

/* Integrate every trajectory from t0 to t1 (eq:rk .. eq:dense), writing
 * y_out at the nodes, y_final, step counts and status, and, when
 * ckpt_every > 0, the checkpoint tape into the workspace.
 *
 * Stiff path (tableau GS_RODAS4 with GS_RHS_KIN3, GS_RHS_KIN8, GS_RHS_ROBER
 * or GS_RHS_HIRES): the
 * Rosenbrock kernel for stiff systems that the paper's library pairs with
 * its explicit kernels (Section "Adaptive explicit Runge--Kutta methods").
 * Each attempt factors (1/(h gamma) I - J) once (LU, partial pivoting) and
 * solves six stages in the method's transformed variables; step control as
 * eq:errnorm / eq:controller with nu = 4 (I control only: beta1 <= 0,
 * beta2 = 0); an attempt whose matrix has a zero or non-finite pivot counts
 * as a NaN error norm.  Not available there (GS_ERR_UNSUPPORTED): a tape,
 * wide groups, gs_solve_vjp, gs_solve_sens, gs_dense_eval.  An explicit
 * tableau with a stiff right-hand side, or GS_RODAS4 with another one, is
 * GS_ERR_UNSUPPORTED as well. */
gs_status gs_solve(const gs_solve_args* args);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): gs_solve
 * without a caller workspace.  Exactly gs_solve's kernels and results; the
 * work-queue counters live in a fixed static device buffer of the library
 * (4 KiB per GPU, held until the process ends) instead of `workspace`, which
 * is ignored.  Forward solves only: ckpt_every must be 0 (a tape would have
 * to outlive the call for gs_solve_vjp, which reads the caller's workspace),
 * else GS_ERR_UNSUPPORTED.  The deferred output records (2 + d) K n doubles
 * are kept in the buffer when they fit ((2 + d) K n <= 480); otherwise
 * GS_DOPRI5 and GS_TSIT5 evaluate their outputs inside the solve kernel (the
 * same values, bit for bit) and GS_VERNER7 is GS_ERR_TOO_LARGE, returned
 * before anything is launched.  Allocates nothing.  Every call on one GPU shares that
 * buffer (the counters are reset by a kernel at the start of each call), so
 * calls that overlap on one GPU -- on different streams, or from different
 * threads without ordering -- race and must not be made. */
gs_status gs_solve_noalloc(const gs_solve_args* args);

/* Longest-first queue order on the device, for gs_solve_args.order (the
 * idle cost of eq:cost falls on the short trajectories that start last).
 * Each trajectory gets a cost key: cost[i] if `cost` (device, [n]) is given,
 * larger first; otherwise a built-in model, the logarithm of the number of
 * dynamical times in the span times rtol^(-1/nu) for the pair's order nu,
 * where a dynamical time is (rc + r_E) / v0 for orbits in the logarithmic
 * halo (r_E: the in-plane radius at the orbit's energy, eq:st-scales) and
 * the span itself stands for it otherwise.  Keys are put in descending order
 * by a counting sort over 65,536 buckets of their range (order within a
 * bucket unspecified; non-finite keys last).  Reads from `args` only rhs,
 * tableau, n, the stream and, for the built-in model, t0, t1, rtol (with
 * their strides) and for the halo y0 and theta.  Writes order [n] (device).
 * Kernels only (no memset, no allocation), so the call can be captured in a
 * graph with the solve.  Workspace: gs_queue_order_workspace_bytes(n),
 * 256-byte aligned, device memory. */
size_t gs_queue_order_workspace_bytes(int64_t n);
gs_status gs_queue_order(const gs_solve_args* args, const double* cost, int64_t* order,
                         void* workspace, size_t workspace_bytes);

/* Reverse-mode derivative of the discrete solution of the last gs_solve call
 * made with the same `fwd` arguments and workspace (tape required): for each
 * trajectory and loss r,
 *   y0bar[r]    = sum_k ybar_out[r][k] S_y0(t_k)    + ybar_final[r] S_y0(t1)
 *   thetabar[r] = sum_k ybar_out[r][k] S_theta(t_k) + ybar_final[r] S_theta(t1)
 * where S are the forward sensitivities of eq:stage-sens along the accepted
 * steps.  In checkpoint mode the segments between checkpoints are
 * recomputed bit-identically; store mode reads every step from the tape.
 * Trajectories whose status is not GS_TRAJ_OK get NaN cotangents. */
gs_status gs_solve_vjp(const gs_solve_args* fwd, const gs_vjp_args* vjp);

/* Forward sensitivities for a gs_solve (eq:sens carried through the
 * stages, eq:stage-sens): M columns, each the derivative of the solution with
 * respect to one input, cols[m] < d for the initial condition y0[cols[m]] or
 * d <= cols[m] < d + p for the parameter theta[cols[m] - d].  In the same
 * launch as the solution (which is written exactly as gs_solve writes it,
 * with the same steps, since step control reads the values only).  Outputs
 * S_final [d][M][n] and, when K > 0, S_out [d][M][K][n]: S[c][m] is
 * d y_c / d input_m; for shared theta (theta_stride 0) it is the derivative
 * of each trajectory with respect to the shared value.  Columns run two per
 * launch.  No tape; queue schedule only.  `wide` runs the head of the order
 * on 16-lane groups as for gs_solve, values and tangents bit-identical to
 * one lane per trajectory.  1 <= M <= 16. */
typedef struct gs_sens_args {
  int32_t M;
  const int32_t* cols;    /* [M], host memory                              */
  double* S_final;        /* [d][M][n]                                     */
  double* S_out;          /* [d][M][K][n], or NULL when K = 0              */
} gs_sens_args;

gs_status gs_solve_sens(const gs_solve_args* args, const gs_sens_args* sens);

/* Profile likelihood of the dark-energy slope (Section "A profile
 * likelihood" and its appendix "Data model and minimiser"): n independent
 * damped Gauss-Newton fits (eq:de-gn) of psi = (Omega_m, h), h = H0 over a
 * reference, at fixed slope lambda[i], for the quintessence system
 * (gs_rhs_quint) with the amplitude a0 solved for flatness E(0) = 1 by
 * Newton steps on the sensitivity S_a0 (the shooting method, eq:de-flat)
 * and the derivative along flat models from the implicit-function theorem
 * (eq:de-ift); both sensitivities come from the same ensemble solve
 * (gs_solve_sens).  Model distances are D_M = (I(0) - I(N_k)) / h and
 * D_H = 1 / (h E(N_k)) in reference Hubble distances at the K nodes.  With
 * K_data = 0 the data sit at the nodes; with K_data > 0 the model at the
 * data e-folds N_data is read off the not-a-knot cubic spline in ln(1+z)
 * through the node values (appendix "Data model and minimiser"; K >= 4, data
 * outside the node range use the end intervals).  Residuals
 * r = (model - data) / sigma, D_M at every data point then D_H.
 *
 * Each iteration: `newton` shooting steps, one solve with both
 * sensitivities at the K nodes, then the update psi <- psi -
 * (J^T J + mu diag J^T J)^{-1} J^T r, scaled back into the box
 * |dOmega_m| <= trust_om, |dh| <= trust_h, and a0 moved by
 * (da0/dOmega_m) dOmega_m.  After the iterations the amplitude is shot again
 * and chi2 (and dist, if given) are evaluated at the returned parameters.
 * All arrays are device memory, trajectory index fastest; the call
 * allocates nothing (workspace: gs_de_profile_workspace_bytes, 256-byte
 * aligned) and only enqueues work on `stream`. */
typedef struct gs_de_profile_args {
  int64_t n;                /* minimisations, <= 2^31                       */
  const double* lambda;     /* [n] fixed slope                              */
  double* omega_m;          /* [n] in: start; out: fitted                   */
  double* h;                /* [n] in: start; out: fitted                   */
  double* a0;               /* [n] in: start amplitude; out: flat amplitude
                               at the fitted parameters                     */
  double omega_r;           /* radiation density (shared)                   */
  int32_t K;                /* nodes, >= 1                                  */
  const double* N_nodes;    /* [K] e-folds N = -ln(1+z), increasing, <= 0   */
  int32_t K_data;           /* data points; 0: the data sit at the nodes     */
  const double* N_data;     /* [K_data] e-folds of the data, or NULL         */
  const double* data;       /* [2][Kd][n] D_M then D_H, Kd = K_data or K     */
  const double* sigma;      /* [2][Kd]                                      */
  int32_t iters;            /* Gauss-Newton iterations                      */
  int32_t newton;           /* shooting steps per iteration                 */
  double mu;                /* damping of eq:de-gn                          */
  double trust_om, trust_h; /* trust box half-widths                        */
  int32_t tableau;          /* gs_tableau_id of the solves                  */
  double N_start;           /* initial e-fold, < 0 (field at rest there)    */
  double rtol, atol;
  double* chi2;             /* [n] out: at the returned parameters          */
  double* chi2_prev;        /* [n] out: before the last update              */
  double* decrement;        /* [n] out: g^T step of the last update         */
  double* dist;             /* [2][Kd][n] out: model distances at the data,
                               or NULL                                      */
  int32_t* status;          /* [n] out: worst gs_traj_status of all solves  */
  void* workspace;
  size_t workspace_bytes;
  void* stream;             /* hipStream_t                                  */
} gs_de_profile_args;

size_t gs_de_profile_workspace_bytes(const gs_de_profile_args* args);
gs_status gs_de_profile(const gs_de_profile_args* args);

/* Solution at arbitrary times t_query [Q][n] (each in [t0, t1]) from the tape
 * of the last gs_solve with `fwd` (eq:dense; replay from the nearest
 * checkpoint, or from t0 when no tape was kept).  y_query is [d][Q][n]. */
gs_status gs_dense_eval(const gs_solve_args* fwd, int32_t Q, const double* t_query,
                        double* y_query, void* stream);

/* Evaluate the right-hand side and its vector-Jacobian product at m points:
 * f = f(t, y, theta) and, for kbar given, ybar = J_y^T kbar,
 * thetabar = J_theta^T kbar.  y, f, ybar, kbar [d][m]; theta, thetabar [p][m];
 * t [m].  ybar, thetabar, kbar may all be NULL.  For the stiff right-hand
 * sides only f is available (a VJP request is GS_ERR_UNSUPPORTED). */
gs_status gs_rhs_eval(int32_t rhs, int64_t m, const double* t, const double* y,
                      const double* theta, double* f, const double* kbar, double* ybar,
                      double* thetabar, void* stream);

/* Graph of one gs_solve: the queue reset and the solve kernel captured once
 * into a hipGraph and replayed with gs_graph_launch on any stream.  The graph
 * keeps the pointers of `args`. */
typedef struct gs_graph gs_graph;
gs_status gs_graph_create(const gs_solve_args* args, gs_graph** out);
gs_status gs_graph_launch(gs_graph* g, void* stream);
void gs_graph_destroy(gs_graph* g);

/* Static description of a status code. */
const char* gs_status_string(gs_status s);

/* Version of this library, e.g. "0.1.0". */
const char* gs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GRADSOLVE_H */
