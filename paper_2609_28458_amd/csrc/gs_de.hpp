// Device steps of the dark-energy profile likelihood (Section "A profile
// likelihood" and its appendix "Data model and minimiser"): one thread per
// minimisation, between ensemble solves with forward sensitivities of the
// quintessence system (y = (phi, u, I), theta = (a0, lambda, Om, Or)).
//
//   E^2(N) = (Om e^{-3N} + Or e^{-4N} + a0 e^{-lambda phi}) / (1 - u^2/6)
//   flatness          g(a0) = E(0)^2 - 1 = 0                     eq:de-flat
//   along flat models da0/dOm = -(dg/dOm)/(dg/da0),
//                     dy/dOm = S_Om + (da0/dOm) S_a0             eq:de-ift
//   distances         D_M = (I(0) - I(N_z)) / h, D_H = 1/(h E(N_z))
//   damped GN         psi <- psi - (J^T J + mu diag J^T J)^{-1} J^T r,
//                     psi = (Om, h), r = (D - data)/sigma        eq:de-gn
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gs {
namespace de {

struct State {
  double phi, u, I;
};

// E^2 = nm / dn at e-fold N, and its total derivative when the state moves
// by (dphi, du), a0 by da0 and Om by dom.
struct E2 {
  double nm, dn, ex;
};
__device__ __forceinline__ E2 e2_at(double N, double phi, double u, double a0, double lam,
                                    double om, double orad) {
  E2 e;
  e.ex = exp(-lam * phi);
  e.nm = om * exp(-3.0 * N) + orad * exp(-4.0 * N) + a0 * e.ex;
  e.dn = 1.0 - u * u * (1.0 / 6.0);
  return e;
}
__device__ __forceinline__ double de2(const E2& e, double N, double u, double a0, double lam,
                                      double dphi, double du, double da0, double dom) {
  const double dnm = exp(-3.0 * N) * dom + e.ex * da0 - lam * a0 * e.ex * dphi;
  const double ddn = -u * du * (1.0 / 3.0);
  return dnm / e.dn - e.nm * ddn / (e.dn * e.dn);
}

// Copy the caller's starting values into theta [4][n] = (a0, lambda, Om, Or).
__global__ void init_kernel(int64_t n, const double* a0, const double* lam, const double* om,
                            double orad, double* theta, int32_t* status_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  theta[i] = a0[i];
  theta[n + i] = lam[i];
  theta[2 * n + i] = om[i];
  theta[3 * n + i] = orad;
  status_out[i] = 0;
}

// One Newton step on g(a0) with the slope from S_a0 at N = 0.
__global__ void shoot_kernel(int64_t n, double* theta, const double* y_final,
                             const double* S_a0, const int32_t* status, int32_t* status_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a0 = theta[i], lam = theta[n + i], om = theta[2 * n + i], orad = theta[3 * n + i];
  const double phi = y_final[i], u = y_final[n + i];
  const E2 e = e2_at(0.0, phi, u, a0, lam, om, orad);
  const double g = e.nm / e.dn - 1.0;
  const double dg = de2(e, 0.0, u, a0, lam, S_a0[i], S_a0[n + i], 1.0, 0.0);
  theta[i] = a0 - g / dg;
  status_out[i] = max(status_out[i], status[i]);
}

// Residuals, Jacobian along flat models and (update != 0) the damped
// Gauss-Newton step of every minimisation.  S_* are [3][2][*][n] with
// column 0 = d/da0 and column 1 = d/dOm.
struct GnArgs {
  int64_t n;
  int32_t K;
  const double* N_nodes;  // [K]
  const double* y_out;    // [3][K][n]
  const double* y_final;  // [3][n]
  const double* S_out;    // [3][2][K][n]
  const double* S_final;  // [3][2][n]
  const double* data;     // [2][K][n]
  const double* sigma;    // [2][K]
  const int32_t* status;  // [n] of the solve
  double mu, trust_om, trust_h;
  int32_t update;
  double* theta;          // [4][n] in/out (a0, Om moved)
  double* h;              // [n] in/out
  double* chi2;           // [n] chi2 at the input parameters
  double* chi2_prev;      // [n] (update) chi2 before this step
  double* decrement;      // [n] (update) g^T step
  double* dist;           // [2][K][n] model distances, or null
  int32_t* status_out;    // [n] worst solver status
};

__global__ void gn_kernel(GnArgs A) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = A.n;
  if (i >= n) return;
  const double a0 = A.theta[i], lam = A.theta[n + i], om = A.theta[2 * n + i];
  const double orad = A.theta[3 * n + i];
  const double h = A.h[i];
  // S layout: component c, column m, [node k,] trajectory
  auto Sf = [&](int c, int m) { return A.S_final[((int64_t)c * 2 + m) * n + i]; };
  auto So = [&](int c, int m, int k) {
    return A.S_out[(((int64_t)c * 2 + m) * A.K + k) * n + i];
  };
  const double phi0 = A.y_final[i], u0 = A.y_final[n + i], I0 = A.y_final[2 * n + i];
  // implicit-function theorem at N = 0
  const E2 e0 = e2_at(0.0, phi0, u0, a0, lam, om, orad);
  const double dg_a0 = de2(e0, 0.0, u0, a0, lam, Sf(0, 0), Sf(1, 0), 1.0, 0.0);
  const double dg_om = de2(e0, 0.0, u0, a0, lam, Sf(0, 1), Sf(1, 1), 0.0, 1.0);
  const double da0 = -dg_om / dg_a0;
  const double dI0 = Sf(2, 1) + da0 * Sf(2, 0);
  double A11 = 0.0, A12 = 0.0, A22 = 0.0, g1 = 0.0, g2 = 0.0, chi2 = 0.0;
  auto add = [&](double D, double dDo, double dDh, double data, double sig, int q, int k) {
    if (A.dist) A.dist[((int64_t)q * A.K + k) * n + i] = D;
    const double r = (D - data) / sig;
    const double j1 = dDo / sig, j2 = dDh / sig;
    A11 += j1 * j1;
    A12 += j1 * j2;
    A22 += j2 * j2;
    g1 += j1 * r;
    g2 += j2 * r;
    chi2 += r * r;
  };
  // D_M at every node, then D_H (the order of the residual vector)
  for (int k = 0; k < A.K; ++k) {
    const double Ik = A.y_out[((int64_t)2 * A.K + k) * n + i];
    const double dIk = So(2, 1, k) + da0 * So(2, 0, k);
    const double DM = (I0 - Ik) / h;
    add(DM, (dI0 - dIk) / h, -DM / h, A.data[(int64_t)k * n + i], A.sigma[k], 0, k);
  }
  for (int k = 0; k < A.K; ++k) {
    const double N = A.N_nodes[k];
    const double phi = A.y_out[(int64_t)k * n + i], u = A.y_out[((int64_t)A.K + k) * n + i];
    const E2 e = e2_at(N, phi, u, a0, lam, om, orad);
    const double E = sqrt(e.nm / e.dn);
    const double DH = 1.0 / (h * E);
    const double dphi = So(0, 1, k) + da0 * So(0, 0, k);
    const double du = So(1, 1, k) + da0 * So(1, 0, k);
    const double dE2 = de2(e, N, u, a0, lam, dphi, du, da0, 1.0);
    add(DH, -0.5 * dE2 / (h * E * E * E), -DH / h, A.data[((int64_t)A.K + k) * n + i],
        A.sigma[A.K + k], 1, k);
  }
  A.chi2[i] = chi2;
  A.status_out[i] = max(A.status_out[i], A.status[i]);
  if (!A.update) return;
  const double B11 = A11 * (1.0 + A.mu), B22 = A22 * (1.0 + A.mu);
  const double det = B11 * B22 - A12 * A12;
  double s1 = (B22 * g1 - A12 * g2) / det;
  double s2 = (B11 * g2 - A12 * g1) / det;
  // back into the trust box |dOm| <= trust_om, |dh| <= trust_h
  const double f = fmin(1.0, fmin(A.trust_om / fmax(fabs(s1), 1e-300),
                                  A.trust_h / fmax(fabs(s2), 1e-300)));
  s1 *= f;
  s2 *= f;
  A.chi2_prev[i] = chi2;
  A.decrement[i] = g1 * s1 + g2 * s2;
  A.theta[2 * n + i] = om - s1;
  A.h[i] = h - s2;
  A.theta[i] = a0 - da0 * s1;  // the amplitude moved to the new Om
}

// Fitted values back to the caller's arrays.
__global__ void finish_kernel(int64_t n, const double* theta, double* a0, double* om) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  a0[i] = theta[i];
  om[i] = theta[2 * n + i];
}

}  // namespace de
}  // namespace gs
