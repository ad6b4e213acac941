// Oracle (test infrastructure only): the stiff path -- an adaptive
// Rosenbrock integrator, one trajectory at a time, plain and slow.
//
// The paper's library ships a Rosenbrock kernel for stiff systems (Section
// "Adaptive explicit Runge-Kutta methods" and the Discussion) without giving
// its method; the reading here is Hairer & Wanner's RODAS (Rodas4, order 4
// with an embedded order-3 estimate, stiffly accurate), written in the
// textbook form of a Rosenbrock method (Hairer & Wanner 1996, Sec. IV.7):
//
//   (I - h gamma J) k_i = h f(y + sum_{j<i} alpha_ij k_j) + h J sum_{j<i} gamma_ij k_j
//   y+ = y + sum_j b_j k_j,   e = sum_j (b_j - bhat_j) k_j,   J = df/dy(y)
//
// for autonomous right-hand sides.  The coefficients are published in the
// transformed variables u_i = sum_{j<=i} gamma_ij k_j (the form that avoids
// the products with J); this file types those and converts them to the form
// above: Gamma = (diag(1/gamma) - C)^{-1}, alpha = A Gamma, b = m Gamma,
// bhat = (m - e) Gamma.  The linear systems are solved by Gaussian
// elimination with partial pivoting.  Step control is that of the explicit
// oracle (eq:errnorm, eq:controller, nu = 4); output times are landed on (the
// step is shortened to end there) instead of interpolated.
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "gso.hpp"

namespace gso {
namespace stiff {

constexpr int S = 6;
constexpr int MD = 8;   // largest stiff state
constexpr int MP = 12;  // most stiff parameters

// Rodas4 in transformed variables (Hairer & Wanner), rows below the diagonal.
constexpr double kGamma = 0.25;
const double kA[15] = {1.544,
                       0.9466785280815826,
                       0.2557011698983284,
                       3.314825187068521,
                       2.896124015972201,
                       0.9986419139977817,
                       1.221224509226641,
                       6.019134481288629,
                       12.53708332932087,
                       -0.6878860361058950,
                       1.221224509226641,
                       6.019134481288629,
                       12.53708332932087,
                       -0.6878860361058950,
                       1.0};
const double kC[15] = {-5.6688,
                       -2.430093356833875,
                       -0.2063599157091915,
                       -0.1073529058151375,
                       -9.594562251023355,
                       -20.47028614809616,
                       7.496443313967647,
                       -10.24680431464352,
                       -33.99990352819905,
                       11.70890893206160,
                       8.083246795921522,
                       -7.981132988064893,
                       -31.52159432874371,
                       16.31930543123136,
                       -6.058818238834054};
const double kM[S] = {1.221224509226641, 6.019134481288629, 12.53708332932087,
                      -0.6878860361058950, 1.0, 1.0};
const double kE[S] = {0.0, 0.0, 0.0, 0.0, 0.0, 1.0};

struct Coeffs {
  double gamma;
  double alpha[S][S], Gam[S][S], b[S], bhat[S];
};

// Standard-form coefficients from the transformed ones.
Coeffs make_coeffs() {
  Coeffs K{};
  K.gamma = kGamma;
  double A[S][S] = {}, Ginv[S][S] = {};
  int q = 0;
  for (int i = 1; i < S; ++i)
    for (int j = 0; j < i; ++j) {
      A[i][j] = kA[q];
      Ginv[i][j] = -kC[q];
      ++q;
    }
  for (int i = 0; i < S; ++i) Ginv[i][i] = 1.0 / kGamma;
  // Gamma = Ginv^{-1}, lower triangular: forward substitution column by column
  for (int c = 0; c < S; ++c) {
    for (int i = 0; i < S; ++i) {
      double acc = (i == c) ? 1.0 : 0.0;
      for (int j = 0; j < i; ++j) acc -= Ginv[i][j] * K.Gam[j][c];
      K.Gam[i][c] = acc / Ginv[i][i];
    }
  }
  for (int i = 0; i < S; ++i)
    for (int c = 0; c < S; ++c) {
      double acc = 0.0;
      for (int j = 0; j < S; ++j) acc += A[i][j] * K.Gam[j][c];
      K.alpha[i][c] = acc;
    }
  for (int c = 0; c < S; ++c) {
    double acc = 0.0, acc2 = 0.0;
    for (int j = 0; j < S; ++j) {
      acc += kM[j] * K.Gam[j][c];
      acc2 += (kM[j] - kE[j]) * K.Gam[j][c];
    }
    K.b[c] = acc;
    K.bhat[c] = acc2;
  }
  return K;
}

const Coeffs& coeffs() {
  static const Coeffs K = make_coeffs();
  return K;
}

// ---------------------------------------------------------------------------
// Stiff mass-action kinetics (stand-ins for the classic stiff chemistry test
// problems; the networks are this library's own).
//
// kin3: y = (a, b, c), theta = (k1, k2, k3)
//   a -> b (k1 a),  b + c -> 2c (k2 b c),  c -> a (k3 c);  a + b + c conserved
// kin8: y1..y8, theta = (k1..k10, s, k12)
//   y1 <-> y2 (k1, k2), y2 -> y3 (k3), y3 <-> y4 (k4, k5),
//   y4 + y5 <-> y6 (k6 y4 y5, k7), y6 -> y7 (k8), y7 -> y8 (k9), y8 -> y1 (k10),
//   source -> y5 (s), y5 -> sink (k12);  y1+y2+y3+y4+y6+y7+y8 conserved
//
// The two classic stiff chemistry problems named with the paper's Rosenbrock
// kernel (Discussion: Robertson 1966; Schaefer 1975), in their standard
// form (Hairer & Wanner 1996, Sec. IV.1 and IV.10), with the rate constants
// as parameters so that an ensemble can draw them:
// rober: y = (y1, y2, y3), theta = (k1, k2, k3), nominal (0.04, 3e7, 1e4)
//   y1' = -k1 y1 + k3 y2 y3
//   y2' =  k1 y1 - k3 y2 y3 - k2 y2^2
//   y3' =  k2 y2^2                          y1 + y2 + y3 conserved
// hires: y1..y8, theta = (a, b, c, s, d, e, kf, g), nominal
//   (1.71, 0.43, 8.32, 0.0007, 0.035, 1.12, 280, 0.69); the problem's other
//   constants are sums of these (8.75 = c + b, 10.03 = c + a, 1.745 = a + d,
//   1.81 = e + g):
//   y1' = -a y1 + b y2 + c y3 + s
//   y2' =  a y1 - (c + b) y2
//   y3' = -(c + a) y3 + b y4 + d y5
//   y4' =  c y2 + a y3 - e y4
//   y5' = -(a + d) y5 + b y6 + b y7
//   y6' = -kf y6 y8 + g y4 + a y5 - b y6 + g y7
//   y7' =  kf y6 y8 - (e + g) y7
//   y8' = -kf y6 y8 + (e + g) y7            y7 + y8 conserved
int dim(int rhs) { return (rhs == RHS_KIN3 || rhs == RHS_ROBER) ? 3 : 8; }
int npar(int rhs) {
  return rhs == RHS_KIN3 ? 3 : rhs == RHS_KIN8 ? 12 : rhs == RHS_ROBER ? 3 : 8;
}
bool is_stiff_rhs(int rhs) {
  return rhs == RHS_KIN3 || rhs == RHS_KIN8 || rhs == RHS_ROBER || rhs == RHS_HIRES;
}

void eval(int rhs, const double* y, const double* k, double* f) {
  if (rhs == RHS_ROBER) {
    const double r1 = k[0] * y[0], r2 = k[1] * y[1] * y[1], r3 = k[2] * y[1] * y[2];
    f[0] = -r1 + r3;
    f[1] = r1 - r3 - r2;
    f[2] = r2;
    return;
  }
  if (rhs == RHS_HIRES) {
    const double a = k[0], b = k[1], c = k[2], s = k[3], d = k[4], e = k[5], kf = k[6],
                 g = k[7];
    const double r = kf * y[5] * y[7];
    f[0] = -a * y[0] + b * y[1] + c * y[2] + s;
    f[1] = a * y[0] - (c + b) * y[1];
    f[2] = -(c + a) * y[2] + b * y[3] + d * y[4];
    f[3] = c * y[1] + a * y[2] - e * y[3];
    f[4] = -(a + d) * y[4] + b * y[5] + b * y[6];
    f[5] = -r + g * y[3] + a * y[4] - b * y[5] + g * y[6];
    f[6] = r - (e + g) * y[6];
    f[7] = -r + (e + g) * y[6];
    return;
  }
  if (rhs == RHS_KIN3) {
    const double r1 = k[0] * y[0], r2 = k[1] * y[1] * y[2], r3 = k[2] * y[2];
    f[0] = -r1 + r3;
    f[1] = r1 - r2;
    f[2] = r2 - r3;
    return;
  }
  double r[12];
  r[0] = k[0] * y[0];
  r[1] = k[1] * y[1];
  r[2] = k[2] * y[1];
  r[3] = k[3] * y[2];
  r[4] = k[4] * y[3];
  r[5] = k[5] * y[3] * y[4];
  r[6] = k[6] * y[5];
  r[7] = k[7] * y[5];
  r[8] = k[8] * y[6];
  r[9] = k[9] * y[7];
  r[10] = k[10];
  r[11] = k[11] * y[4];
  f[0] = -r[0] + r[1] + r[9];
  f[1] = r[0] - r[1] - r[2];
  f[2] = r[2] - r[3] + r[4];
  f[3] = r[3] - r[4] - r[5] + r[6];
  f[4] = -r[5] + r[6] + r[10] - r[11];
  f[5] = r[5] - r[6] - r[7];
  f[6] = r[7] - r[8];
  f[7] = r[8] - r[9];
}

// J[i][j] = d f_i / d y_j, written out by hand.
void jac(int rhs, const double* y, const double* k, double J[MD][MD]) {
  const int d = dim(rhs);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) J[i][j] = 0.0;
  if (rhs == RHS_ROBER) {
    J[0][0] = -k[0];
    J[0][1] = k[2] * y[2];
    J[0][2] = k[2] * y[1];
    J[1][0] = k[0];
    J[1][1] = -k[2] * y[2] - 2.0 * k[1] * y[1];
    J[1][2] = -k[2] * y[1];
    J[2][1] = 2.0 * k[1] * y[1];
    return;
  }
  if (rhs == RHS_HIRES) {
    const double a = k[0], b = k[1], c = k[2], dd = k[4], e = k[5], kf = k[6], g = k[7];
    J[0][0] = -a;
    J[0][1] = b;
    J[0][2] = c;
    J[1][0] = a;
    J[1][1] = -(c + b);
    J[2][2] = -(c + a);
    J[2][3] = b;
    J[2][4] = dd;
    J[3][1] = c;
    J[3][2] = a;
    J[3][3] = -e;
    J[4][4] = -(a + dd);
    J[4][5] = b;
    J[4][6] = b;
    J[5][3] = g;
    J[5][4] = a;
    J[5][5] = -kf * y[7] - b;
    J[5][6] = g;
    J[5][7] = -kf * y[5];
    J[6][5] = kf * y[7];
    J[6][6] = -(e + g);
    J[6][7] = kf * y[5];
    J[7][5] = -kf * y[7];
    J[7][6] = e + g;
    J[7][7] = -kf * y[5];
    return;
  }
  if (rhs == RHS_KIN3) {
    J[0][0] = -k[0];
    J[0][2] = k[2];
    J[1][0] = k[0];
    J[1][1] = -k[1] * y[2];
    J[1][2] = -k[1] * y[1];
    J[2][1] = k[1] * y[2];
    J[2][2] = k[1] * y[1] - k[2];
    return;
  }
  J[0][0] = -k[0];
  J[0][1] = k[1];
  J[0][7] = k[9];
  J[1][0] = k[0];
  J[1][1] = -k[1] - k[2];
  J[2][1] = k[2];
  J[2][2] = -k[3];
  J[2][3] = k[4];
  J[3][2] = k[3];
  J[3][3] = -k[4] - k[5] * y[4];
  J[3][4] = -k[5] * y[3];
  J[3][5] = k[6];
  J[4][3] = -k[5] * y[4];
  J[4][4] = -k[5] * y[3] - k[11];
  J[4][5] = k[6];
  J[5][3] = k[5] * y[4];
  J[5][4] = k[5] * y[3];
  J[5][5] = -k[6] - k[7];
  J[6][5] = k[7];
  J[6][6] = -k[8];
  J[7][6] = k[8];
  J[7][7] = -k[9];
}

// ---------------------------------------------------------------------------
// Gaussian elimination with partial pivoting (first row of largest |entry|),
// factors in place: rows swapped whole, multipliers below the diagonal.
// Returns false if a pivot is zero or not finite.
bool lu(int d, double M[MD][MD], int piv[MD]) {
  for (int k = 0; k < d; ++k) {
    int p = k;
    for (int r = k + 1; r < d; ++r)
      if (std::fabs(M[r][k]) > std::fabs(M[p][k])) p = r;
    piv[k] = p;
    if (p != k)
      for (int c = 0; c < d; ++c) std::swap(M[k][c], M[p][c]);
    if (!(std::fabs(M[k][k]) > 0.0) || !std::isfinite(M[k][k])) return false;
    for (int r = k + 1; r < d; ++r) {
      const double l = M[r][k] / M[k][k];
      M[r][k] = l;
      for (int c = k + 1; c < d; ++c) M[r][c] -= l * M[k][c];
    }
  }
  return true;
}

void lu_solve(int d, const double M[MD][MD], const int piv[MD], double* x) {
  for (int k = 0; k < d; ++k) std::swap(x[k], x[piv[k]]);
  for (int r = 1; r < d; ++r)
    for (int c = 0; c < r; ++c) x[r] -= M[r][c] * x[c];
  for (int r = d - 1; r >= 0; --r) {
    for (int c = r + 1; c < d; ++c) x[r] -= M[r][c] * x[c];
    x[r] /= M[r][r];
  }
}

double err_norm(int d, const double* e, const double* y, const double* yn, double rtol,
                double atol) {
  double acc = 0.0;
  for (int j = 0; j < d; ++j) {
    const double sj = atol + rtol * std::max(std::fabs(y[j]), std::fabs(yn[j]));
    const double r = e[j] / sj;
    acc += r * r;
  }
  return std::sqrt(acc / d);
}

// Starting step of Hairer, Norsett & Wanner (1993, Sec. II.4) with exponent
// 1/4, as in the explicit oracle.
double initial_step(int rhs, int d, double t0, double t1, const double* y0, const double* f0,
                    const double* th, double rtol, double atol) {
  const double span = t1 - t0;
  double d0 = 0.0, d1 = 0.0;
  for (int j = 0; j < d; ++j) {
    const double sc = atol + std::fabs(y0[j]) * rtol;
    d0 += (y0[j] / sc) * (y0[j] / sc);
    d1 += (f0[j] / sc) * (f0[j] / sc);
  }
  d0 = std::sqrt(d0 / d);
  d1 = std::sqrt(d1 / d);
  double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
  h0 = std::min(h0, span);
  double y1[MD], f1[MD];
  for (int j = 0; j < d; ++j) y1[j] = y0[j] + h0 * f0[j];
  eval(rhs, y1, th, f1);
  double d2 = 0.0;
  for (int j = 0; j < d; ++j) {
    const double sc = atol + std::fabs(y0[j]) * rtol;
    const double r = (f1[j] - f0[j]) / sc;
    d2 += r * r;
  }
  d2 = std::sqrt(d2 / d) / h0;
  double h1;
  if (d1 <= 1e-15 && d2 <= 1e-15)
    h1 = std::max(1e-6, h0 * 1e-3);
  else
    h1 = std::pow(0.01 / std::max(d1, d2), 1.0 / 4.0);
  return std::min(std::min(100.0 * h0, h1), span);
}

void solve_one(const gso_problem& P, int64_t i) {
  const Coeffs& K = coeffs();
  const int d = dim(P.rhs), p = npar(P.rhs);
  const int64_t n = P.n;
  double y[MD], th[MP];
  for (int c = 0; c < d; ++c) y[c] = P.y0[(int64_t)c * n + i];
  for (int c = 0; c < p; ++c)
    th[c] = P.theta_stride ? P.theta[(int64_t)c * P.theta_stride + i] : P.theta[c];
  const double t0 = P.t0[P.t_stride ? i : 0];
  const double t1 = P.t1[P.t_stride ? i : 0];
  const double rtol = P.rtol[P.tol_stride ? i : 0];
  const double atol = P.atol[P.tol_stride ? i : 0];
  auto node_t = [&](int kk) {
    return P.t_out_stride ? P.t_out[(int64_t)kk * P.t_out_stride + i] : P.t_out[kk];
  };
  auto store = [&](int kk, const double* v) {
    for (int c = 0; c < d; ++c) P.y_out[((int64_t)c * P.K + kk) * n + i] = v[c];
  };
  int32_t nacc = 0, nrej = 0, status = ST_OK;
  int kp = 0;
  while (kp < P.K && node_t(kp) <= t0) store(kp++, y);
  bool y0fin = true;
  for (int c = 0; c < d; ++c) y0fin = y0fin && std::isfinite(y[c]);
  if (!y0fin) status = ST_NONFINITE;
  if (y0fin && t1 > t0) {
    double f0[MD];
    eval(P.rhs, y, th, f0);
    double t = t0;
    double h = P.h0 > 0.0 ? std::min(P.h0, t1 - t0)
                          : initial_step(P.rhs, d, t0, t1, y, f0, th, rtol, atol);
    int nan_streak = 0;
    for (;;) {
      if ((int64_t)nacc + nrej >= P.max_steps) {
        status = ST_MAX_STEPS;
        break;
      }
      // the next stop is the next output time, or t1
      const double stop = kp < P.K ? node_t(kp) : t1;
      bool land = false;
      if (t + h >= stop) {
        h = stop - t;
        land = true;
      }
      double J[MD][MD], M[MD][MD];
      jac(P.rhs, y, th, J);
      for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) M[r][c] = (r == c ? 1.0 : 0.0) - h * K.gamma * J[r][c];
      int piv[MD];
      const bool ok = lu(d, M, piv);
      double k[S][MD];
      for (int s = 0; s < S && ok; ++s) {
        double Y[MD], g[MD], fY[MD], x[MD];
        for (int c = 0; c < d; ++c) {
          double ay = 0.0, ag = 0.0;
          for (int j = 0; j < s; ++j) {
            ay += K.alpha[s][j] * k[j][c];
            ag += K.Gam[s][j] * k[j][c];
          }
          Y[c] = y[c] + ay;
          g[c] = ag;
        }
        if (s == 0)
          for (int c = 0; c < d; ++c) fY[c] = f0[c];
        else
          eval(P.rhs, Y, th, fY);
        for (int r = 0; r < d; ++r) {
          double jg = 0.0;
          for (int c = 0; c < d; ++c) jg += J[r][c] * g[c];
          x[r] = h * fY[r] + h * jg;
        }
        lu_solve(d, M, piv, x);
        for (int c = 0; c < d; ++c) k[s][c] = x[c];
      }
      double yn[MD], e[MD];
      double en = NAN;
      if (ok) {
        for (int c = 0; c < d; ++c) {
          double acc = 0.0, ae = 0.0;
          for (int j = 0; j < S; ++j) {
            acc += K.b[j] * k[j][c];
            ae += (K.b[j] - K.bhat[j]) * k[j][c];
          }
          yn[c] = y[c] + acc;
          e[c] = ae;
        }
        en = err_norm(d, e, y, yn, rtol, atol);
      }
      const bool finite = std::isfinite(en);
      const bool accept = finite && en <= 1.0;
      double factor;
      if (!finite)
        factor = P.alpha_min;
      else if (en == 0.0)
        factor = P.alpha_max;
      else
        factor = std::min(P.alpha_max, std::max(P.alpha_min, P.safety * std::pow(en, -0.25)));
      if (accept) {
        ++nacc;
        t = land ? stop : t + h;
        for (int c = 0; c < d; ++c) y[c] = yn[c];
        bool yfin = true;
        for (int c = 0; c < d; ++c) yfin = yfin && std::isfinite(y[c]);
        if (!yfin) {
          status = ST_NONFINITE;
          break;
        }
        while (kp < P.K && node_t(kp) <= t) store(kp++, y);
        eval(P.rhs, y, th, f0);
        nan_streak = 0;
        if (t >= t1) break;
      } else {
        ++nrej;
        if (!finite) {
          if (++nan_streak >= 50) {
            status = ST_NONFINITE;
            break;
          }
        } else {
          nan_streak = 0;
        }
      }
      h = h * factor;
      if (std::fabs(h) < 16.0 * 2.220446049250313e-16 * std::max(std::fabs(t), 1.0)) {
        status = ST_DT_UNDERFLOW;
        break;
      }
    }
  }
  for (; kp < P.K; ++kp) {
    double nanv[MD];
    for (int c = 0; c < d; ++c) nanv[c] = std::nan("");
    store(kp, nanv);
  }
  for (int c = 0; c < d; ++c) P.y_final[(int64_t)c * n + i] = y[c];
  P.n_acc[i] = nacc;
  P.n_rej[i] = nrej;
  P.status[i] = status;
}

}  // namespace stiff
}  // namespace gso

extern "C" {

int gso_stiff_solve(const gso_problem* P) {
  using namespace gso;
  if (!P || P->n < 0 || !stiff::is_stiff_rhs(P->rhs) || P->tableau != RODAS4 ||
      P->m != 0 || P->h_replay || P->h_cap)
    return 1;
  int nt = P->nthreads > 0 ? P->nthreads : 1;
  if (nt > P->n) nt = (int)std::max<int64_t>(P->n, 1);
  auto work = [&](int w) {
    for (int64_t i = w; i < P->n; i += nt) stiff::solve_one(*P, i);
  };
  if (nt == 1) {
    work(0);
  } else {
    std::vector<std::thread> th;
    for (int w = 0; w < nt; ++w) th.emplace_back(work, w);
    for (auto& x : th) x.join();
  }
  return 0;
}

// f and the analytic Jacobian J [d][d] (row-major) of a stiff right-hand side.
int gso_stiff_rhs(int rhs, const double* y, const double* theta, double* f, double* J) {
  using namespace gso;
  if (!stiff::is_stiff_rhs(rhs)) return 1;
  const int d = stiff::dim(rhs);
  stiff::eval(rhs, y, theta, f);
  double Jm[stiff::MD][stiff::MD];
  stiff::jac(rhs, y, theta, Jm);
  for (int r = 0; r < d; ++r)
    for (int c = 0; c < d; ++c) J[r * d + c] = Jm[r][c];
  return 0;
}

// Standard-form Rodas4 coefficients: gamma, alpha [6][6], Gamma [6][6]
// (diagonal gamma), b [6], bhat [6], written in that order to out[1 + 36 + 36 + 12].
int gso_rodas4(double* out) {
  using namespace gso::stiff;
  const Coeffs& K = coeffs();
  int o = 0;
  out[o++] = K.gamma;
  for (int i = 0; i < S; ++i)
    for (int j = 0; j < S; ++j) out[o++] = K.alpha[i][j];
  for (int i = 0; i < S; ++i)
    for (int j = 0; j < S; ++j) out[o++] = K.Gam[i][j];
  for (int j = 0; j < S; ++j) out[o++] = K.b[j];
  for (int j = 0; j < S; ++j) out[o++] = K.bhat[j];
  return 0;
}

}  // extern "C"
