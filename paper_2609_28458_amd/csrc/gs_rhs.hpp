// Right-hand sides f(t, y, theta) of the ensembles, with hand-written
// vector-Jacobian products for the discrete adjoint.
//
// Each system is a struct with
//   D, P                 state and parameter counts
//   Par prep(theta)      per-trajectory constants derived from theta (done
//                        once per trajectory, kept in registers)
//   f(t, y, par, dy)     the right-hand side
// prep and f are templates on the scalar type: double, or the forward-mode
// ad::Dual of the sensitivity kernels (ParT<Dual> carries d par / d theta).
//   vjp(t, y, theta, par, kb, yb, thb)
//                        yb = J_y^T kb (overwritten), thb += J_theta^T kb
// All loops have compile-time trip counts so arrays stay in VGPRs.
#pragma once

#include <hip/hip_runtime.h>

#include "gs_dual.hpp"

namespace gs {

// 1/x from the hardware reciprocal refined by two Newton steps (error within
// about one ulp; not always the correctly rounded quotient).  A third of the
// instructions of an IEEE division and a shorter dependency chain.
__device__ __forceinline__ double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// 1/x with one Newton step (relative error ~2e-15): for the scales of the
// error norm, which only decide acceptance.
__device__ __forceinline__ double fast_rcp1(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

namespace ad {
// d(1/x) = -x' / x^2, with the value of the double version.
template <int M>
__device__ __forceinline__ Dual<M> fast_rcp(const Dual<M>& x) {
  Dual<M> r;
  r.v = gs::fast_rcp(x.v);
  const double g = -r.v * r.v;
#pragma unroll
  for (int m = 0; m < M; ++m) r.d[m] = g * x.d[m];
  return r;
}
}  // namespace ad

// ---------------------------------------------------------------------------
// Harmonic oscillator: x' = v, v' = -omega^2 x.  Closed-form test system.
struct Harmonic {
  static constexpr int D = 2, P = 1;
  template <class T>
  struct ParT { T w2; };
  using Par = ParT<double>;
  template <class T>
  __device__ static ParT<T> prep(const T (&th)[P]) { return ParT<T>{th[0] * th[0]}; }
  template <class T>
  __device__ static void f(double, const T (&y)[D], const ParT<T>& p, T (&dy)[D]) {
    dy[0] = y[1];
    dy[1] = -p.w2 * y[0];
  }
  __device__ static void vjp(double, const double (&y)[D], const double (&th)[P], const Par& p,
                             const double (&kb)[D], double (&yb)[D], double (&thb)[P]) {
    yb[0] = -p.w2 * kb[1];
    yb[1] = kb[0];
    thb[0] += -2.0 * th[0] * y[0] * kb[1];
  }
};

// ---------------------------------------------------------------------------
// Planar Kepler problem: r'' = -mu r / |r|^3.  Closed-form test system.
struct Kepler {
  static constexpr int D = 4, P = 1;
  template <class T>
  struct ParT { T mu; };
  using Par = ParT<double>;
  template <class T>
  __device__ static ParT<T> prep(const T (&th)[P]) { return ParT<T>{th[0]}; }
  template <class T>
  __device__ static void f(double, const T (&y)[D], const ParT<T>& p, T (&dy)[D]) {
    const T r2 = y[0] * y[0] + y[1] * y[1];
    const T ir3 = fast_rcp(r2 * sqrt(r2));
    dy[0] = y[2];
    dy[1] = y[3];
    dy[2] = -p.mu * ir3 * y[0];
    dy[3] = -p.mu * ir3 * y[1];
  }
  __device__ static void vjp(double, const double (&y)[D], const double (&)[P], const Par& p,
                             const double (&kb)[D], double (&yb)[D], double (&thb)[P]) {
    // a = -mu r / r^3;  da/dr = -mu (I / r^3 - 3 r r^T / r^5)  (symmetric)
    const double r2 = y[0] * y[0] + y[1] * y[1];
    const double ir3 = fast_rcp(r2 * sqrt(r2));
    const double ir5 = ir3 * fast_rcp(r2);
    const double rw = y[0] * kb[2] + y[1] * kb[3];
    yb[0] = -p.mu * (ir3 * kb[2] - 3.0 * ir5 * rw * y[0]);
    yb[1] = -p.mu * (ir3 * kb[3] - 3.0 * ir5 * rw * y[1]);
    yb[2] = kb[0];
    yb[3] = kb[1];
    thb[0] += -ir3 * rw;
  }
};

// ---------------------------------------------------------------------------
// Test particle in the flattened logarithmic halo (eq:loghalo):
//   Phi = (v0^2/2) ln(rc^2 + R^2 + z^2/q^2),  x'' = -grad Phi.
// With g = (x, y, z/q^2) and D = rc^2 + x^2 + y^2 + z^2/q^2 the acceleration
// is a = -(v0^2 / D) g.
struct LogHalo {
  static constexpr int D = 6, P = 3;
  template <class T>
  struct ParT { T v02, iq2, rc2; };
  using Par = ParT<double>;
  template <class T>
  __device__ static ParT<T> prep(const T (&th)[P]) {
    const T iq = 1.0 / th[1];
    return ParT<T>{th[0] * th[0], iq * iq, th[2] * th[2]};
  }
  template <class T>
  __device__ static void f(double, const T (&y)[D], const ParT<T>& p, T (&dy)[D]) {
    const T Dn = fma(y[2] * y[2], p.iq2, fma(y[1], y[1], fma(y[0], y[0], p.rc2)));
    const T s = -p.v02 * fast_rcp(Dn);
    dy[0] = y[3];
    dy[1] = y[4];
    dy[2] = y[5];
    dy[3] = s * y[0];
    dy[4] = s * y[1];
    dy[5] = s * (p.iq2 * y[2]);
  }
  __device__ static void vjp(double, const double (&y)[D], const double (&th)[P], const Par& p,
                             const double (&kb)[D], double (&yb)[D], double (&thb)[P]) {
    const double Dn = fma(y[2] * y[2], p.iq2, fma(y[1], y[1], fma(y[0], y[0], p.rc2)));
    const double inv = fast_rcp(Dn);
    const double s = -p.v02 * inv;
    const double gz = p.iq2 * y[2];
    // w = kb[3..5] is the cotangent of the acceleration.
    const double gw = y[0] * kb[3] + y[1] * kb[4] + gz * kb[5];
    // da/dpos = s (diag(1, 1, 1/q^2) - 2 g g^T / D)
    const double c = -2.0 * s * inv * gw;
    yb[0] = s * kb[3] + c * y[0];
    yb[1] = s * kb[4] + c * y[1];
    yb[2] = s * p.iq2 * kb[5] + c * gz;
    yb[3] = kb[0];
    yb[4] = kb[1];
    yb[5] = kb[2];
    // da/dv0 = 2 a / v0;  da/drc = -2 rc s g / D;
    // da/dq = (2 s / q^3) z (z g / D - e_z)
    const double v0 = th[0], q = th[1], rc = th[2];
    thb[0] += -2.0 * v0 * inv * gw;
    thb[2] += -2.0 * rc * s * inv * gw;
    const double iq3 = p.iq2 / q;
    thb[1] += 2.0 * s * iq3 * y[2] * (y[2] * gw * inv - kb[5]);
  }
};

// ---------------------------------------------------------------------------
// Orbit-averaged spin precession in the orbital velocity v (eq:prec-spins,
// eq:prec-L, eq:prec-omega, eq:prec-rr; G = c = M = 1).
//   y = (Lhat, S1hat, S2hat), theta = (q, chi1, chi2),
//   m1 = 1/(1+q), m2 = q/(1+q), eta = m1 m2, S_j = chi_j m_j^2, L = eta / v,
//   Omega_1 = (v^6/2) [(4+3q) L Lhat + S2 S2hat - 3 (S2 L.S2hat + q S1 L.S1hat) Lhat],
//   Omega_2 = the same with 1 <-> 2 and q -> 1/q,
//   dS_j/dt = Omega_j x S_j,  dL/dt = -(v/eta) sum_j S_j dS_j/dt,
//   dv/dt = (32/5) eta v^9 (1 + b2 v^2 + b3 v^3 + b4 v^4),
// with the 2PN terms b2 = -(743/336 + 11 eta/4), b3 = 4 pi - beta,
// b4 = 34103/18144 + 13661 eta/2016 + 59 eta^2/18 + sigma,
//   beta  = (1/12) sum_j chi_j (L.S_j) (113 m_j^2 + 75 eta),
//   sigma = (eta/48) chi1 chi2 (721 (L.S1)(L.S2) - 247 S1.S2).
// f = (dL/dt, dS1/dt, dS2/dt) / (dv/dt).
struct SpinPrec {
  static constexpr int D = 9, P = 3;
  template <class T>
  struct ParT {
    T q, iq, eta, ieta, S1, S2, cq1, cq2, c1, c2, sig, b2, b4c;
    // Products of the above that f folds into its coefficients:
    // -3 q S1, -3 S2, -3 S1, -3 S2 / q, 721 sig, -247 sig, (64/5) eta,
    // (4 + 3q) eta, (4 + 3/q) eta, -S1/eta, -S2/eta.
    T m3qS1, m3S2, m3S1, m3iqS2, sig721, sig247, k128e, cq1e, cq2e, mS1e, mS2e;
  };
  using Par = ParT<double>;
  template <class T>
  __device__ static ParT<T> prep(const T (&th)[P]) {
    ParT<T> p;
    const T q = th[0], chi1 = th[1], chi2 = th[2];
    const T m1 = 1.0 / (1.0 + q);
    const T m2 = q * m1;
    p.q = q;
    p.iq = 1.0 / q;
    p.eta = m1 * m2;
    p.ieta = 1.0 / p.eta;
    p.S1 = chi1 * m1 * m1;
    p.S2 = chi2 * m2 * m2;
    p.cq1 = 4.0 + 3.0 * q;
    p.cq2 = 4.0 + 3.0 * p.iq;
    p.c1 = chi1 * (113.0 * m1 * m1 + 75.0 * p.eta) * (1.0 / 12.0);
    p.c2 = chi2 * (113.0 * m2 * m2 + 75.0 * p.eta) * (1.0 / 12.0);
    p.sig = p.eta * chi1 * chi2 * (1.0 / 48.0);
    p.b2 = -(743.0 / 336.0 + 2.75 * p.eta);
    p.b4c = 34103.0 / 18144.0 + (13661.0 / 2016.0) * p.eta + (59.0 / 18.0) * p.eta * p.eta;
    p.m3qS1 = -3.0 * (q * p.S1);
    p.m3S2 = -3.0 * p.S2;
    p.m3S1 = -3.0 * p.S1;
    p.m3iqS2 = -3.0 * (p.S2 * p.iq);
    p.sig721 = 721.0 * p.sig;
    p.sig247 = -247.0 * p.sig;
    p.k128e = 12.8 * p.eta;
    p.cq1e = p.cq1 * p.eta;
    p.cq2e = p.cq2 * p.eta;
    p.mS1e = -(p.S1 * p.ieta);
    p.mS2e = -(p.S2 * p.ieta);
    return p;
  }

  // Shared forward pieces, also needed by the VJP (powers of v are plain
  // doubles, everything else follows the scalar type).
  template <class T>
  struct FwdT {
    double v2, v3, v4, v6h, k9;
    T L, Ls1, Ls2, s12, cL1, cL2;
    T Om1[3], Om2[3], ds1[3], ds2[3], u[3], poly, r;
  };
  using Fwd = FwdT<double>;
  template <class T>
  __device__ static void forward(double v, const T (&y)[D], const ParT<T>& p, FwdT<T>& w) {
    w.v2 = v * v;
    w.v3 = w.v2 * v;
    w.v4 = w.v2 * w.v2;
    const double v6 = w.v3 * w.v3;
    w.v6h = 0.5 * v6;
    // Every multiply-add of the expressions below is one fused operation
    // (the same arithmetic, about a third fewer instructions): dot products
    // and the spin-weighted sums as chains of fma, cross products as
    // fma(a, b, -c d), the radiation-reaction polynomial by Horner's rule.
    w.L = p.eta * fast_rcp(v);
    w.Ls1 = fma(y[2], y[5], fma(y[1], y[4], y[0] * y[3]));
    w.Ls2 = fma(y[2], y[8], fma(y[1], y[7], y[0] * y[6]));
    w.s12 = fma(y[5], y[8], fma(y[4], y[7], y[3] * y[6]));
    w.cL1 = fma(p.cq1, w.L, -3.0 * fma(p.S2, w.Ls2, p.q * p.S1 * w.Ls1));
    w.cL2 = fma(p.cq2, w.L, -3.0 * fma(p.S1, w.Ls1, p.S2 * w.Ls2 * p.iq));
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      w.Om1[i] = w.v6h * fma(w.cL1, y[i], p.S2 * y[6 + i]);
      w.Om2[i] = w.v6h * fma(w.cL2, y[i], p.S1 * y[3 + i]);
    }
    w.ds1[0] = fma(w.Om1[1], y[5], -(w.Om1[2] * y[4]));
    w.ds1[1] = fma(w.Om1[2], y[3], -(w.Om1[0] * y[5]));
    w.ds1[2] = fma(w.Om1[0], y[4], -(w.Om1[1] * y[3]));
    w.ds2[0] = fma(w.Om2[1], y[8], -(w.Om2[2] * y[7]));
    w.ds2[1] = fma(w.Om2[2], y[6], -(w.Om2[0] * y[8]));
    w.ds2[2] = fma(w.Om2[0], y[7], -(w.Om2[1] * y[6]));
#pragma unroll
    for (int i = 0; i < 3; ++i) w.u[i] = fma(p.S1, w.ds1[i], p.S2 * w.ds2[i]);
    const T beta = fma(p.c1, w.Ls1, p.c2 * w.Ls2);
    const T sigma = p.sig * fma(721.0 * w.Ls1, w.Ls2, -247.0 * w.s12);
    w.poly = fma(p.b4c + sigma, w.v4, fma(4.0 * M_PI - beta, w.v3, fma(p.b2, w.v2, 1.0)));
    w.k9 = 6.4 * v6 * w.v3;  // (32/5) v^9
    w.r = fast_rcp(w.k9 * p.eta * w.poly);
  }
  // The right-hand side itself: the function of forward() with every
  // constant factor folded into prepared coefficients, and with
  // v^6 / (2 dv/dt) = 1 / ((64/5) eta v^3 poly) folded into the two
  // precession coefficients, so the precession vectors, and with them the
  // cross products, come out already divided by dv/dt; the polynomial of
  // dv/dt by Horner's rule in v.  The same function up to rounding, with
  // about a third fewer multiplies.  The adjoint differentiates forward().
  template <class T>
  __device__ static void f(double v, const T (&y)[D], const ParT<T>& p, T (&dy)[D]) {
    const double v2 = v * v;
    const double rv = fast_rcp(v);
    const T Ls1 = fma(y[2], y[5], fma(y[1], y[4], y[0] * y[3]));
    const T Ls2 = fma(y[2], y[8], fma(y[1], y[7], y[0] * y[6]));
    const T s12 = fma(y[5], y[8], fma(y[4], y[7], y[3] * y[6]));
    const T cL1 = fma(p.cq1e, rv, fma(p.m3S2, Ls2, p.m3qS1 * Ls1));
    const T cL2 = fma(p.cq2e, rv, fma(p.m3S1, Ls1, p.m3iqS2 * Ls2));
    const T beta = fma(p.c1, Ls1, p.c2 * Ls2);
    const T sigma = fma(p.sig721 * Ls1, Ls2, p.sig247 * s12);
    const T poly = fma(fma(fma(p.b4c + sigma, v, 4.0 * M_PI - beta), v, p.b2), v2, 1.0);
    const T gr = fast_rcp(((p.k128e * v) * v2) * poly);
    const T A1 = gr * cL1, B1 = gr * p.S2;
    const T A2 = gr * cL2, B2 = gr * p.S1;
    T Om1[3], Om2[3], ds1[3], ds2[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Om1[i] = fma(A1, y[i], B1 * y[6 + i]);
      Om2[i] = fma(A2, y[i], B2 * y[3 + i]);
    }
    ds1[0] = fma(Om1[1], y[5], -(Om1[2] * y[4]));
    ds1[1] = fma(Om1[2], y[3], -(Om1[0] * y[5]));
    ds1[2] = fma(Om1[0], y[4], -(Om1[1] * y[3]));
    ds2[0] = fma(Om2[1], y[8], -(Om2[2] * y[7]));
    ds2[1] = fma(Om2[2], y[6], -(Om2[0] * y[8]));
    ds2[2] = fma(Om2[0], y[7], -(Om2[1] * y[6]));
    const T cS1 = v * p.mS1e, cS2 = v * p.mS2e;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      dy[i] = fma(cS1, ds1[i], cS2 * ds2[i]);
      dy[3 + i] = ds1[i];
      dy[6 + i] = ds2[i];
    }
  }
  __device__ static void vjp(double v, const double (&y)[D], const double (&th)[P], const Par& p,
                             const double (&kb)[D], double (&yb)[D], double (&thb)[P]) {
    Fwd w;
    forward(v, y, p, w);
    // g = (dL, ds1, ds2) with dL = -(v/eta) u; f = r g.
    const double nve = -v * p.ieta;
    double gb[9];
    double rb = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      gb[i] = kb[i] * w.r;
      gb[3 + i] = kb[3 + i] * w.r;
      gb[6 + i] = kb[6 + i] * w.r;
      rb += kb[i] * (nve * w.u[i]) + kb[3 + i] * w.ds1[i] + kb[6 + i] * w.ds2[i];
    }
    // r = 1 / (k9 eta poly)
    const double dvdtb = -rb * w.r * w.r;
    double etab = dvdtb * w.k9 * w.poly;
    const double polyb = dvdtb * w.k9 * p.eta;
    const double b2b = polyb * w.v2;
    const double betab = -polyb * w.v3;
    const double b4cb = polyb * w.v4;
    const double sigmab = polyb * w.v4;
    // sigma = sig (721 Ls1 Ls2 - 247 s12)
    const double sigb = sigmab * (721.0 * w.Ls1 * w.Ls2 - 247.0 * w.s12);
    double Ls1b = sigmab * p.sig * 721.0 * w.Ls2;
    double Ls2b = sigmab * p.sig * 721.0 * w.Ls1;
    const double s12b = -247.0 * sigmab * p.sig;
    // beta = c1 Ls1 + c2 Ls2
    const double c1b = betab * w.Ls1;
    const double c2b = betab * w.Ls2;
    Ls1b += betab * p.c1;
    Ls2b += betab * p.c2;
    // dL = nve u, u = S1 ds1 + S2 ds2
    double ub[3];
    double uu = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      ub[i] = nve * gb[i];
      uu += w.u[i] * gb[i];
    }
    etab += v * p.ieta * p.ieta * uu;  // d(-v/eta)/deta = v / eta^2
    double ds1b[3], ds2b[3];
    double S1b = 0.0, S2b = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      ds1b[i] = gb[3 + i] + p.S1 * ub[i];
      ds2b[i] = gb[6 + i] + p.S2 * ub[i];
      S1b += w.ds1[i] * ub[i];
      S2b += w.ds2[i] * ub[i];
    }
    // ds1 = Om1 x s1: Om1b = s1 x ds1b, s1b += ds1b x Om1 (same for 2)
    double Om1b[3], Om2b[3], Lb[3], s1b[3], s2b[3];
    Om1b[0] = y[4] * ds1b[2] - y[5] * ds1b[1];
    Om1b[1] = y[5] * ds1b[0] - y[3] * ds1b[2];
    Om1b[2] = y[3] * ds1b[1] - y[4] * ds1b[0];
    Om2b[0] = y[7] * ds2b[2] - y[8] * ds2b[1];
    Om2b[1] = y[8] * ds2b[0] - y[6] * ds2b[2];
    Om2b[2] = y[6] * ds2b[1] - y[7] * ds2b[0];
    s1b[0] = ds1b[1] * w.Om1[2] - ds1b[2] * w.Om1[1];
    s1b[1] = ds1b[2] * w.Om1[0] - ds1b[0] * w.Om1[2];
    s1b[2] = ds1b[0] * w.Om1[1] - ds1b[1] * w.Om1[0];
    s2b[0] = ds2b[1] * w.Om2[2] - ds2b[2] * w.Om2[1];
    s2b[1] = ds2b[2] * w.Om2[0] - ds2b[0] * w.Om2[2];
    s2b[2] = ds2b[0] * w.Om2[1] - ds2b[1] * w.Om2[0];
    // Om1 = v6h (cL1 Lhat + S2 s2);  Om2 = v6h (cL2 Lhat + S1 s1)
    double cL1b = 0.0, cL2b = 0.0, o1s2 = 0.0, o2s1 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cL1b += Om1b[i] * y[i];
      cL2b += Om2b[i] * y[i];
      o1s2 += Om1b[i] * y[6 + i];
      o2s1 += Om2b[i] * y[3 + i];
    }
    cL1b *= w.v6h;
    cL2b *= w.v6h;
    S2b += w.v6h * o1s2;
    S1b += w.v6h * o2s1;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Lb[i] = w.v6h * (w.cL1 * Om1b[i] + w.cL2 * Om2b[i]);
      s2b[i] += w.v6h * p.S2 * Om1b[i];
      s1b[i] += w.v6h * p.S1 * Om2b[i];
    }
    // cL1 = cq1 L - 3 (S2 Ls2 + q S1 Ls1)
    const double cq1b = cL1b * w.L;
    double Lmagb = cL1b * p.cq1;
    S2b += -3.0 * cL1b * w.Ls2;
    Ls2b += -3.0 * cL1b * p.S2;
    double qb = -3.0 * cL1b * p.S1 * w.Ls1;
    S1b += -3.0 * cL1b * p.q * w.Ls1;
    Ls1b += -3.0 * cL1b * p.q * p.S1;
    // cL2 = cq2 L - 3 (S1 Ls1 + S2 Ls2 / q)
    const double cq2b = cL2b * w.L;
    Lmagb += cL2b * p.cq2;
    S1b += -3.0 * cL2b * w.Ls1;
    Ls1b += -3.0 * cL2b * p.S1;
    S2b += -3.0 * cL2b * w.Ls2 * p.iq;
    Ls2b += -3.0 * cL2b * p.S2 * p.iq;
    const double iqb = -3.0 * cL2b * p.S2 * w.Ls2;
    // dot products
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Lb[i] += Ls1b * y[3 + i] + Ls2b * y[6 + i];
      s1b[i] += Ls1b * y[i] + s12b * y[6 + i];
      s2b[i] += Ls2b * y[i] + s12b * y[3 + i];
    }
    // L = eta / v
    etab += Lmagb * fast_rcp(v);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      yb[i] = Lb[i];
      yb[3 + i] = s1b[i];
      yb[6 + i] = s2b[i];
    }
    // Parameter constants -> (q, chi1, chi2).
    const double q = th[0], chi1 = th[1], chi2 = th[2];
    const double m1 = 1.0 / (1.0 + q);
    const double m2 = q * m1;
    const double m1s = m1 * m1;
    const double deta = m1s * (m1 - m2);  // d eta / d q
    const double dm1 = -m1s, dm2 = m1s;   // d m_j / d q
    const double A1 = 113.0 * m1s + 75.0 * p.eta;
    const double A2 = 113.0 * m2 * m2 + 75.0 * p.eta;
    etab += b2b * (-2.75) + b4cb * (13661.0 / 2016.0 + (118.0 / 18.0) * p.eta);
    etab += sigb * chi1 * chi2 * (1.0 / 48.0);
    qb += etab * deta;
    qb += S1b * (2.0 * chi1 * m1 * dm1) + S2b * (2.0 * chi2 * m2 * dm2);
    qb += iqb * (-p.iq * p.iq) + cq1b * 3.0 + cq2b * (-3.0 * p.iq * p.iq);
    qb += c1b * chi1 * (226.0 * m1 * dm1 + 75.0 * deta) * (1.0 / 12.0);
    qb += c2b * chi2 * (226.0 * m2 * dm2 + 75.0 * deta) * (1.0 / 12.0);
    thb[0] += qb;
    thb[1] += S1b * m1s + c1b * A1 * (1.0 / 12.0) + sigb * p.eta * chi2 * (1.0 / 48.0);
    thb[2] += S2b * m2 * m2 + c2b * A2 * (1.0 / 12.0) + sigb * p.eta * chi1 * (1.0 / 48.0);
  }
};

// ---------------------------------------------------------------------------
// Thawing quintessence, V = V0 exp(-lambda phi), in e-folds N (eq:de-model,
// eq:de-rhs).  y = (phi, u, I), theta = (a0, lambda, Omega_m, Omega_r):
//   v = a0 e^{-lambda phi},  E^2 = (Om e^{-3N} + Or e^{-4N} + v) / (1 - u^2/6),
//   dlnE/dN = -(3 Om e^{-3N} + 4 Or e^{-4N}) / (2 E^2) - u^2/2,
//   phi' = u,  u' = -(3 + dlnE/dN) u + 3 lambda v / E^2,  I' = e^{-N} / E.
struct Quint {
  static constexpr int D = 3, P = 4;
  template <class T>
  struct ParT { T a0, lam, om, orad; };
  using Par = ParT<double>;
  template <class T>
  __device__ static ParT<T> prep(const T (&th)[P]) { return ParT<T>{th[0], th[1], th[2], th[3]}; }
  template <class T>
  __device__ static void f(double N, const T (&y)[D], const ParT<T>& p, T (&dy)[D]) {
    const double eN = exp(-N);
    const double e3 = eN * eN * eN;
    const double e4 = e3 * eN;
    const T u = y[1];
    const T pot = p.a0 * exp(-p.lam * y[0]);
    const T den = 1.0 - u * u * (1.0 / 6.0);
    const T iE2 = den * fast_rcp(p.om * e3 + p.orad * e4 + pot);
    const T dlnE = -0.5 * (3.0 * p.om * e3 + 4.0 * p.orad * e4) * iE2 - 0.5 * u * u;
    dy[0] = u;
    dy[1] = -(3.0 + dlnE) * u + 3.0 * p.lam * pot * iE2;
    dy[2] = eN * sqrt(iE2);
  }
  __device__ static void vjp(double N, const double (&y)[D], const double (&)[P], const Par& p,
                             const double (&kb)[D], double (&yb)[D], double (&thb)[P]) {
    const double eN = exp(-N);
    const double e3 = eN * eN * eN;
    const double e4 = e3 * eN;
    const double u = y[1];
    const double ex = exp(-p.lam * y[0]);
    const double pot = p.a0 * ex;
    const double den = 1.0 - u * u * (1.0 / 6.0);
    const double Bg = p.om * e3 + p.orad * e4;
    const double iS = fast_rcp(Bg + pot);
    const double iE2 = den * iS;
    const double Cc = 3.0 * p.om * e3 + 4.0 * p.orad * e4;
    const double dlnE = -0.5 * Cc * iE2 - 0.5 * u * u;
    // f1 = -(3 + dlnE) u + 3 lam pot iE2
    double ub = kb[0] + kb[1] * (-(3.0 + dlnE));
    const double dlnEb = -kb[1] * u;
    double lamb = kb[1] * 3.0 * pot * iE2;
    double potb = kb[1] * 3.0 * p.lam * iE2;
    double iE2b = kb[1] * 3.0 * p.lam * pot;
    // f2 = eN iE2^(1/2)
    const double sq = sqrt(iE2);
    iE2b += kb[2] * eN * 0.5 * fast_rcp(sq);
    // dlnE = -0.5 Cc iE2 - 0.5 u^2
    const double Ccb = -0.5 * dlnEb * iE2;
    iE2b += -0.5 * dlnEb * Cc;
    ub += -dlnEb * u;
    // iE2 = den / (Bg + pot)
    const double denb = iE2b * iS;
    const double sumb = -iE2b * den * iS * iS;
    potb += sumb;
    ub += denb * (-u * (1.0 / 3.0));
    // Bg, Cc
    const double omb = sumb * e3 + Ccb * 3.0 * e3;
    const double orb = sumb * e4 + Ccb * 4.0 * e4;
    // pot = a0 exp(-lam phi)
    const double a0b = potb * ex;
    lamb += potb * pot * (-y[0]);
    const double phib = potb * pot * (-p.lam);
    yb[0] = phib;
    yb[1] = ub;
    yb[2] = 0.0;
    thb[0] += a0b;
    thb[1] += lamb;
    thb[2] += omb;
    thb[3] += orb;
  }
};

}  // namespace gs
