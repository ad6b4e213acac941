// Oracle (test infrastructure only): forward-mode dual numbers.
//
// The paper obtains the right-hand side of the sensitivity equations by
// forward-mode automatic differentiation of f (Section "Derivatives",
// equation eq:sens and eq:stage-sens).  This file is that forward mode, in
// its plainest form: a value plus a gradient vector of runtime length m.
// A constant has m = 0 (all partials zero).
#pragma once
#include <cmath>

namespace gso {

constexpr int MAXM = 16;

struct Dual {
  double v;
  int m;
  double g[MAXM];
  Dual() : v(0.0), m(0) {}
  Dual(double x) : v(x), m(0) {}  // NOLINT: implicit constant promotion
};

inline double gpart(const Dual& a, int i) { return i < a.m ? a.g[i] : 0.0; }
inline int mmax(const Dual& a, const Dual& b) { return a.m > b.m ? a.m : b.m; }

inline Dual operator+(const Dual& a, const Dual& b) {
  Dual r(a.v + b.v);
  r.m = mmax(a, b);
  for (int i = 0; i < r.m; ++i) r.g[i] = gpart(a, i) + gpart(b, i);
  return r;
}
inline Dual operator-(const Dual& a, const Dual& b) {
  Dual r(a.v - b.v);
  r.m = mmax(a, b);
  for (int i = 0; i < r.m; ++i) r.g[i] = gpart(a, i) - gpart(b, i);
  return r;
}
inline Dual operator-(const Dual& a) {
  Dual r(-a.v);
  r.m = a.m;
  for (int i = 0; i < r.m; ++i) r.g[i] = -a.g[i];
  return r;
}
inline Dual operator*(const Dual& a, const Dual& b) {
  Dual r(a.v * b.v);
  r.m = mmax(a, b);
  for (int i = 0; i < r.m; ++i) r.g[i] = gpart(a, i) * b.v + a.v * gpart(b, i);
  return r;
}
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r(a.v / b.v);
  r.m = mmax(a, b);
  for (int i = 0; i < r.m; ++i)
    r.g[i] = (gpart(a, i) * b.v - a.v * gpart(b, i)) / (b.v * b.v);
  return r;
}
inline Dual& operator+=(Dual& a, const Dual& b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, const Dual& b) { a = a - b; return a; }
inline Dual& operator*=(Dual& a, const Dual& b) { a = a * b; return a; }

inline Dual sqrt(const Dual& a) {
  Dual r(std::sqrt(a.v));
  r.m = a.m;
  for (int i = 0; i < r.m; ++i) r.g[i] = a.g[i] / (2.0 * r.v);
  return r;
}
inline Dual exp(const Dual& a) {
  Dual r(std::exp(a.v));
  r.m = a.m;
  for (int i = 0; i < r.m; ++i) r.g[i] = a.g[i] * r.v;
  return r;
}
inline Dual log(const Dual& a) {
  Dual r(std::log(a.v));
  r.m = a.m;
  for (int i = 0; i < r.m; ++i) r.g[i] = a.g[i] / a.v;
  return r;
}

// A dual variable seeded with unit partial in direction `dir`.
inline Dual seed(double x, int m, int dir) {
  Dual r(x);
  r.m = m;
  for (int i = 0; i < m; ++i) r.g[i] = (i == dir) ? 1.0 : 0.0;
  return r;
}

inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }

}  // namespace gso
