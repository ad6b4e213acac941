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
// Optionally the model distances at the data redshifts are read off a cubic
// spline through the node values (appendix "Data model and minimiser"): the
// not-a-knot spline in ln(1+z), built here in N = -ln(1+z) (an affine change
// of variable maps the one spline onto the other), applied as a fixed matrix
// W [Kd][K] to the node values and to their derivatives.
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

// Spline weights: thread c interpolates the unit vector e_c.  Slopes s_i of
// the Hermite form solve the tridiagonal system of a C2 cubic spline, with
// the not-a-knot conditions (third derivative continuous at the second and
// the next-to-last node) folded into the first and last rows; Thomas
// elimination.  Data outside the node range use the end intervals.  K >= 4,
// u strictly increasing; tmp holds 3 K doubles per thread.
__global__ void spline_weights_kernel(int32_t K, const double* u, int32_t Kd, const double* ud,
                                      double* tmp, double* W) {
  const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (c >= K) return;
  double* cp = tmp + (size_t)c * 3 * K;
  double* rp = cp + K;
  double* s = rp + K;
  auto hh = [&](int i) { return u[i + 1] - u[i]; };
  auto yv = [&](int i) { return i == c ? 1.0 : 0.0; };
  auto dl = [&](int i) { return (yv(i + 1) - yv(i)) / hh(i); };
  for (int i = 0; i < K; ++i) {
    double a, b, cc, r;
    if (i == 0) {
      const double h0 = hh(0), h1 = hh(1);
      a = 0.0;
      b = h1;
      cc = h0 + h1;
      r = ((3.0 * h0 + 2.0 * h1) * h1 * dl(0) + h0 * h0 * dl(1)) / (h0 + h1);
    } else if (i == K - 1) {
      const double hl = hh(K - 2), hm = hh(K - 3);
      a = hl + hm;
      b = hm;
      cc = 0.0;
      r = (hl * hl * dl(K - 3) + (3.0 * hl + 2.0 * hm) * hm * dl(K - 2)) / (hm + hl);
    } else {
      const double hm = hh(i - 1), hi = hh(i);
      a = hi;
      b = 2.0 * (hm + hi);
      cc = hm;
      r = 3.0 * (hi * dl(i - 1) + hm * dl(i));
    }
    const double m = i == 0 ? b : b - a * cp[i - 1];
    cp[i] = cc / m;
    rp[i] = i == 0 ? r / m : (r - a * rp[i - 1]) / m;
  }
  s[K - 1] = rp[K - 1];
  for (int i = K - 2; i >= 0; --i) s[i] = rp[i] - cp[i] * s[i + 1];
  for (int q = 0; q < Kd; ++q) {
    const double x = ud[q];
    int i = 0;
    while (i < K - 2 && x > u[i + 1]) ++i;
    const double h = hh(i);
    const double tt = (x - u[i]) / h;
    const double t2 = tt * tt, t3 = t2 * tt;
    W[(size_t)q * K + c] = yv(i) * (2.0 * t3 - 3.0 * t2 + 1.0) + h * s[i] * (t3 - 2.0 * t2 + tt) +
                           yv(i + 1) * (3.0 * t2 - 2.0 * t3) + h * s[i + 1] * (t3 - t2);
  }
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
  const double* data;     // [2][Kd][n]
  const double* sigma;    // [2][Kd]
  int32_t Kd;             // data points (= K without spline)
  const double* W;        // [Kd][K] spline weights, or null: data at the nodes
  const int32_t* status;  // [n] of the solve
  double mu, trust_om, trust_h;
  int32_t update;
  double* theta;          // [4][n] in/out (a0, Om moved)
  double* h;              // [n] in/out
  double* chi2;           // [n] chi2 at the input parameters
  double* chi2_prev;      // [n] (update) chi2 before this step
  double* decrement;      // [n] (update) g^T step
  double* dist;           // [2][Kd][n] model distances at the data, or null
  int32_t* status_out;    // [n] worst solver status
};

__global__ void __launch_bounds__(256) gn_kernel(GnArgs A) {
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
  auto add = [&](double D, double dDo, int q, int j) {
    if (A.dist) A.dist[((int64_t)q * A.Kd + j) * n + i] = D;
    const double sig = A.sigma[q * A.Kd + j];
    const double r = (D - A.data[((int64_t)q * A.Kd + j) * n + i]) / sig;
    const double j1 = dDo / sig, j2 = (-D / h) / sig;  // distances scale as 1/h
    A11 += j1 * j1;
    A12 += j1 * j2;
    A22 += j2 * j2;
    g1 += j1 * r;
    g2 += j2 * r;
    chi2 += r * r;
  };
  // D_M and D_H at node k with their derivatives along flat models
  auto node_dm = [&](int k, double& dDo) {
    const double Ik = A.y_out[((int64_t)2 * A.K + k) * n + i];
    const double dIk = So(2, 1, k) + da0 * So(2, 0, k);
    dDo = (dI0 - dIk) / h;
    return (I0 - Ik) / h;
  };
  auto node_dh = [&](int k, double& dDo) {
    const double N = A.N_nodes[k];
    const double phi = A.y_out[(int64_t)k * n + i], u = A.y_out[((int64_t)A.K + k) * n + i];
    const E2 e = e2_at(N, phi, u, a0, lam, om, orad);
    const double E = sqrt(e.nm / e.dn);
    const double dphi = So(0, 1, k) + da0 * So(0, 0, k);
    const double du = So(1, 1, k) + da0 * So(1, 0, k);
    const double dE2 = de2(e, N, u, a0, lam, dphi, du, da0, 1.0);
    dDo = -0.5 * dE2 / (h * E * E * E);
    return 1.0 / (h * E);
  };
  // D_M at every data point, then D_H (the order of the residual vector)
  if (!A.W) {
#pragma unroll 4
    for (int k = 0; k < A.K; ++k) {
      double d;
      const double D = node_dm(k, d);
      add(D, d, 0, k);
    }
#pragma unroll 4
    for (int k = 0; k < A.K; ++k) {
      double d;
      const double D = node_dh(k, d);
      add(D, d, 1, k);
    }
  } else {
    // One pass over the nodes per chunk of data points, the spline sums of
    // the chunk in registers (the weights are the same for every fit).
    constexpr int kChunk = 8;
    for (int j0 = 0; j0 < A.Kd; j0 += kChunk) {
      double sD[2][kChunk], sd[2][kChunk];
#pragma unroll
      for (int jj = 0; jj < kChunk; ++jj) sD[0][jj] = sD[1][jj] = sd[0][jj] = sd[1][jj] = 0.0;
      // unrolled so the loads of several nodes are in flight together
#pragma unroll 8
      for (int k = 0; k < A.K; ++k) {
        double d0, d1;
        const double DM = node_dm(k, d0);
        const double DH = node_dh(k, d1);
#pragma unroll
        for (int jj = 0; jj < kChunk; ++jj) {
          if (j0 + jj < A.Kd) {
            const double w = A.W[(int64_t)(j0 + jj) * A.K + k];
            sD[0][jj] = fma(w, DM, sD[0][jj]);
            sd[0][jj] = fma(w, d0, sd[0][jj]);
            sD[1][jj] = fma(w, DH, sD[1][jj]);
            sd[1][jj] = fma(w, d1, sd[1][jj]);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int jj = 0; jj < kChunk; ++jj)
          if (j0 + jj < A.Kd) add(sD[q][jj], sd[q][jj], q, j0 + jj);
    }
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
