// Oracle (test infrastructure only): right-hand sides f(t, y, theta),
// templated on the scalar so the same text gives values (double) and, with
// gso::Dual, the forward-mode products J_y S + df/dtheta of eq:sens.
// Parity unpinned: the spin-orbit (beta) and spin-spin (sigma) terms of the
// precession's radiation-reaction polynomial, which the paper does not
// print; everything else here has a pin of its own.
#pragma once
#include <cmath>

#include "dual.hpp"

namespace gso {

using std::exp;
using std::log;
using std::sqrt;

// Harmonic oscillator (closed-form test system): y = (x, v), theta = (omega).
template <class T>
void f_harmonic(double, const T* y, const T* th, T* dy) {
  dy[0] = y[1];
  dy[1] = -(th[0] * th[0]) * y[0];
}

// Planar Kepler problem (closed-form test system): y = (x, y, vx, vy),
// theta = (mu); acceleration -mu r / |r|^3.
template <class T>
void f_kepler(double, const T* y, const T* th, T* dy) {
  T r2 = y[0] * y[0] + y[1] * y[1];
  T r3 = r2 * sqrt(r2);
  dy[0] = y[2];
  dy[1] = y[3];
  dy[2] = -th[0] * y[0] / r3;
  dy[3] = -th[0] * y[1] / r3;
}

// Test particle in the flattened logarithmic halo, eq:loghalo:
// Phi = (v0^2 / 2) ln(rc^2 + R^2 + z^2 / q^2), x'' = -grad Phi.
// y = (x, y, z, vx, vy, vz), theta = (v0, q, rc).
template <class T>
void f_loghalo(double, const T* y, const T* th, T* dy) {
  const T& v0 = th[0];
  const T& q = th[1];
  const T& rc = th[2];
  T D = rc * rc + y[0] * y[0] + y[1] * y[1] + (y[2] * y[2]) / (q * q);
  T s = -(v0 * v0) / D;
  dy[0] = y[3];
  dy[1] = y[4];
  dy[2] = y[5];
  dy[3] = s * y[0];
  dy[4] = s * y[1];
  dy[5] = s * y[2] / (q * q);
}

// Orbit-averaged spin precession in the orbital velocity v (Section "Spin
// precession": eq:prec-spins, eq:prec-L, eq:prec-omega, eq:prec-rr), units
// G = c = M = 1.  y = (Lhat, S1hat, S2hat), theta = (q, chi1, chi2).
// Radiation reaction: the paper leaves the b_k to the precession package;
// this oracle uses the 2PN terms (b2, b3 with spin-orbit beta, b4 with
// spin-spin sigma; b5..b7 = 0), a reading the design notes record.
template <class T>
void f_spinprec(double v, const T* y, const T* th, T* dy) {
  const T& q = th[0];
  const T& chi1 = th[1];
  const T& chi2 = th[2];
  T m1 = T(1.0) / (T(1.0) + q);
  T m2 = q / (T(1.0) + q);
  T eta = m1 * m2;
  T S1 = chi1 * m1 * m1;
  T S2 = chi2 * m2 * m2;
  T L = eta / v;
  const T* Lh = y;
  const T* s1 = y + 3;
  const T* s2 = y + 6;
  T Ls1 = Lh[0] * s1[0] + Lh[1] * s1[1] + Lh[2] * s1[2];
  T Ls2 = Lh[0] * s2[0] + Lh[1] * s2[1] + Lh[2] * s2[2];
  T s12 = s1[0] * s2[0] + s1[1] * s2[1] + s1[2] * s2[2];
  double v6h = 0.5 * std::pow(v, 6);
  // eq:prec-omega and its 1 <-> 2, q -> 1/q image.
  T cL1 = (T(4.0) + T(3.0) * q) * L - T(3.0) * (S2 * Ls2 + q * S1 * Ls1);
  T cL2 = (T(4.0) + T(3.0) / q) * L - T(3.0) * (S1 * Ls1 + S2 * Ls2 / q);
  T Om1[3], Om2[3];
  for (int i = 0; i < 3; ++i) {
    Om1[i] = v6h * (cL1 * Lh[i] + S2 * s2[i]);
    Om2[i] = v6h * (cL2 * Lh[i] + S1 * s1[i]);
  }
  T ds1[3], ds2[3], dL[3];
  ds1[0] = Om1[1] * s1[2] - Om1[2] * s1[1];
  ds1[1] = Om1[2] * s1[0] - Om1[0] * s1[2];
  ds1[2] = Om1[0] * s1[1] - Om1[1] * s1[0];
  ds2[0] = Om2[1] * s2[2] - Om2[2] * s2[1];
  ds2[1] = Om2[2] * s2[0] - Om2[0] * s2[2];
  ds2[2] = Om2[0] * s2[1] - Om2[1] * s2[0];
  for (int i = 0; i < 3; ++i) dL[i] = -(v / eta) * (S1 * ds1[i] + S2 * ds2[i]);
  // eq:prec-rr with the 2PN coefficients.  beta and sigma have no pin of
  // their own (parity unpinned): only the paper's printed attempt counts and
  // angle errors, which depend on them weakly, check them.
  const double pi = 3.14159265358979323846;
  T beta = (chi1 * Ls1 * (T(113.0) * m1 * m1 + T(75.0) * eta) +
            chi2 * Ls2 * (T(113.0) * m2 * m2 + T(75.0) * eta)) / T(12.0);
  T sigma = eta / T(48.0) * chi1 * chi2 * (T(721.0) * Ls1 * Ls2 - T(247.0) * s12);
  T b2 = -(T(743.0 / 336.0) + T(11.0 / 4.0) * eta);
  T b3 = T(4.0 * pi) - beta;
  T b4 = T(34103.0 / 18144.0) + T(13661.0 / 2016.0) * eta + T(59.0 / 18.0) * eta * eta + sigma;
  T dvdt = T(32.0 / 5.0) * eta * std::pow(v, 9) *
           (T(1.0) + b2 * (v * v) + b3 * (v * v * v) + b4 * (v * v * v * v));
  for (int i = 0; i < 3; ++i) {
    dy[i] = dL[i] / dvdt;
    dy[3 + i] = ds1[i] / dvdt;
    dy[6 + i] = ds2[i] / dvdt;
  }
}

// Thawing quintessence with V = V0 exp(-lambda phi) in e-folds N
// (eq:de-model with the closed-form right-hand side eq:de-rhs).
// y = (phi, u, I), theta = (a0, lambda, Omega_m, Omega_r).
template <class T>
void f_quint(double N, const T* y, const T* th, T* dy) {
  const T& a0 = th[0];
  const T& lam = th[1];
  const T& Om = th[2];
  const T& Orad = th[3];
  const T& phi = y[0];
  const T& u = y[1];
  double e3 = std::exp(-3.0 * N);
  double e4 = std::exp(-4.0 * N);
  T pot = a0 * exp(-lam * phi);                               // v(phi)
  T E2 = (Om * e3 + Orad * e4 + pot) / (T(1.0) - u * u / T(6.0));  // Friedmann
  T dlnE = -(T(3.0) * Om * e3 + T(4.0) * Orad * e4) / (T(2.0) * E2) - u * u / T(2.0);
  dy[0] = u;
  // v'(phi) = -lambda v, so -3 v'/E^2 = +3 lambda v / E^2.
  dy[1] = -(T(3.0) + dlnE) * u + T(3.0) * lam * pot / E2;
  dy[2] = T(std::exp(-N)) / sqrt(E2);
}

template <class T>
void rhs_eval(int id, double t, const T* y, const T* th, T* dy) {
  switch (id) {
    case 0: f_harmonic(t, y, th, dy); break;
    case 1: f_kepler(t, y, th, dy); break;
    case 2: f_loghalo(t, y, th, dy); break;
    case 3: f_spinprec(t, y, th, dy); break;
    default: f_quint(t, y, th, dy); break;
  }
}

}  // namespace gso
