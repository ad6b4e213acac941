// Oracle (test infrastructure only) -- plain, slow, obviously correct FP64
// reference for the adaptive explicit Runge-Kutta ensemble solve of the paper
// (Appendix "Numerical details": eq:rk, eq:errnorm, eq:controller, eq:dense,
// eq:stage-sens).  Only the test suite, the smoke check and the CPU-baseline
// leg of the benchmark may load it; the product library never does, and the
// two share no source.
//
// Compiled with -O2 -fno-fast-math -ffp-contract=off so every operation is
// the rounded IEEE operation written in the source.
#pragma once
#include <cstdint>

namespace gso {

constexpr int MAXS = 10;  // most stages of any tableau (Verner 7)
constexpr int MAXD = 9;   // largest state (spin precession)
constexpr int MAXP = 4;   // most parameters (quintessence)

enum TableauId { DOPRI5 = 0, TSIT5 = 1, VERNER7 = 2, RODAS4 = 3 };
enum DenseKind { DENSE_POLY = 0, DENSE_SHORT_STEP = 1 };

struct Tableau {
  int s;           // stages
  int order;       // nu: order of the propagated solution
  bool fsal;       // last stage evaluated at (t+h, y+) and reused as next k1
  int dense;       // DenseKind
  int deg;         // degree of the dense polynomials b_j(sigma) (DENSE_POLY)
  double c[MAXS];
  double a[MAXS][MAXS];
  double b[MAXS];
  double bdiff[MAXS];     // b_j - bhat_j (eq:rk error weights)
  double P[MAXS][8];      // b_j(sigma) = sum_k P[j][k] sigma^(k+1)
};

const Tableau& tableau(int id);

enum RhsId { RHS_HARMONIC = 0, RHS_KEPLER = 1, RHS_LOGHALO = 2, RHS_SPINPREC = 3, RHS_QUINT = 4,
             RHS_KIN3 = 5, RHS_KIN8 = 6, RHS_ROBER = 7, RHS_HIRES = 8 };
// the last four: stiff chemistry, Rodas4 only
int rhs_dim(int id);     // d
int rhs_nparam(int id);  // p

enum TrajStatus { ST_OK = 0, ST_MAX_STEPS = 1, ST_DT_UNDERFLOW = 2, ST_NONFINITE = 3 };

}  // namespace gso

extern "C" {

// One ensemble problem with host pointers.  Layouts (structure of arrays):
//   y0 [d][n]; theta [p][theta_stride] (stride 0: one vector for all);
//   t0, t1 [t_stride]; rtol, atol [tol_stride]; t_out [K][t_out_stride];
//   y_out [d][K][n]; y_final [d][n]; n_acc, n_rej, status [n].
// Forward sensitivities (m > 0): column c of S is d y / d z_c with z_c the
// initial-condition component cols[c] (< d) or parameter cols[c] - d.
//   S_out [d][m][K][n]; S_final [d][m][n].
// Step record / replay: h_rec [n][h_cap] receives the accepted step sizes;
// if h_replay is given ([n][h_cap], with n_replay[i] entries for trajectory
// i) the adaptive controller is bypassed and exactly those steps are taken
// (frozen-step mode, used for finite differences of the discrete map).
typedef struct {
  int32_t rhs, tableau;
  int64_t n;
  const double* y0;
  const double* theta;
  int64_t theta_stride;
  const double* t0;
  const double* t1;
  int64_t t_stride;
  const double* rtol;
  const double* atol;
  int64_t tol_stride;
  int32_t K;
  const double* t_out;
  int64_t t_out_stride;
  double* y_out;
  double* y_final;
  int32_t* n_acc;
  int32_t* n_rej;
  int32_t* status;
  int64_t max_steps;
  double h0;  // <= 0: starting-step rule
  double safety, alpha_min, alpha_max, beta1, beta2;  // beta1 <= 0: 1/nu
  int32_t no_grow_after_reject;  // 1: cap factor at 1 on the accept after a reject
  int32_t nthreads;
  int32_t m;
  const int32_t* cols;
  double* S_out;
  double* S_final;
  int64_t h_cap;
  double* h_rec;
  const double* h_replay;
  const int32_t* n_replay;
} gso_problem;

int gso_solve(const gso_problem* p);

// Tableau export for the order-condition tests: writes s, order, fsal,
// dense kind and degree to ints[5], then c[s], a[s*s], b[s], bdiff[s],
// P[s*8] to dbl.
int gso_tableau(int id, int32_t* ints, double* dbl);

// f(t, y, theta) at one point; with m > 0 also the Jacobian columns
// d f / d z_c for the same column convention as gso_problem (J [d][m]).
int gso_rhs(int rhs, double t, const double* y, const double* theta, int32_t m,
            const int32_t* cols, double* f, double* J);

// Stiff path (stiff.cpp): Rosenbrock solve of an ensemble of RHS_KIN3 /
// RHS_KIN8 problems with tableau RODAS4 (no sensitivities, no replay);
// outputs are landed on.  f and analytic Jacobian J [d][d] of those
// right-hand sides; standard-form Rodas4 coefficients.
int gso_stiff_solve(const gso_problem* p);
int gso_stiff_rhs(int rhs, const double* y, const double* theta, double* f, double* J);
int gso_rodas4(double* out);
}
