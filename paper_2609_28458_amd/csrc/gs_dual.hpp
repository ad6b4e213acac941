// Forward-mode scalar for the sensitivity kernels: a value and M tangent
// components, the derivative of the value with respect to M seeded inputs
// (initial conditions or parameters).  Every operation computes its value
// with exactly the double operation it replaces, so a sensitivity solve
// takes the same steps, bit for bit, as the plain solve; tangents follow the
// chain rule of that operation, which is eq:sens applied to the discrete
// stages (eq:stage-sens).
//
// The type and its functions live in gs::ad: calls with a Dual argument find
// them by argument-dependent lookup, while unqualified calls on doubles keep
// resolving to the ordinary functions.
#pragma once

#include <hip/hip_runtime.h>

namespace gs {
namespace ad {

template <int M>
struct Dual {
  double v;
  double d[M];
};

// Number of tangent columns of a scalar type (0 for double).
template <class T>
struct width {
  static constexpr int value = 0;
};
template <int M>
struct width<Dual<M>> {
  static constexpr int value = M;
};

template <int M>
__device__ __forceinline__ Dual<M> constant(double x) {
  Dual<M> r;
  r.v = x;
#pragma unroll
  for (int m = 0; m < M; ++m) r.d[m] = 0.0;
  return r;
}

// c ? a : b, component by component (a select of whole structs would make
// the compiler pick between their addresses and keep both in memory).
__device__ __forceinline__ double select(bool c, double a, double b) { return c ? a : b; }
template <int M>
__device__ __forceinline__ Dual<M> select(bool c, const Dual<M>& a, const Dual<M>& b) {
  Dual<M> r;
  r.v = c ? a.v : b.v;
#pragma unroll
  for (int m = 0; m < M; ++m) r.d[m] = c ? a.d[m] : b.d[m];
  return r;
}

__device__ __forceinline__ double val(double x) { return x; }
template <int M>
__device__ __forceinline__ double val(const Dual<M>& x) {
  return x.v;
}

template <int M>
__device__ __forceinline__ Dual<M> operator-(const Dual<M>& a) {
  Dual<M> r;
  r.v = -a.v;
#pragma unroll
  for (int m = 0; m < M; ++m) r.d[m] = -a.d[m];
  return r;
}
template <int M>
__device__ __forceinline__ Dual<M> operator+(const Dual<M>& a, const Dual<M>& b) {
  Dual<M> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int m = 0; m < M; ++m) r.d[m] = a.d[m] + b.d[m];
  return r;
}
template <int M>
__device__ __forceinline__ Dual<M> operator+(const Dual<M>& a, double b) {
  Dual<M> r = a;
  r.v = a.v + b;
  return r;
}
template <int M>
__device__ __forceinline__ Dual<M> operator+(double a, const Dual<M>& b) {
  Dual<M> r = b;
  r.v = a + b.v;
  return r;
}
template <int M>
__device__ __forceinline__ Dual<M> operator-(const Dual<M>& a, const Dual<M>& b) {
  Dual<M> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int m = 0; m < M; ++m) r.d[m] = a.d[m] - b.d[m];
  return r;
}
template <int M>
__device__ __forceinline__ Dual<M> operator-(const Dual<M>& a, double b) {
  Dual<M> r = a;
  r.v = a.v - b;
  return r;
}
template <int M>
__device__ __forceinline__ Dual<M> operator-(double a, const Dual<M>& b) {
  Dual<M> r;
  r.v = a - b.v;
#pragma unroll
  for (int m = 0; m < M; ++m) r.d[m] = -b.d[m];
  return r;
}
template <int M>
__device__ __forceinline__ Dual<M> operator*(const Dual<M>& a, const Dual<M>& b) {
  Dual<M> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int m = 0; m < M; ++m) r.d[m] = ::fma(a.d[m], b.v, a.v * b.d[m]);
  return r;
}
template <int M>
__device__ __forceinline__ Dual<M> operator*(const Dual<M>& a, double b) {
  Dual<M> r;
  r.v = a.v * b;
#pragma unroll
  for (int m = 0; m < M; ++m) r.d[m] = a.d[m] * b;
  return r;
}
template <int M>
__device__ __forceinline__ Dual<M> operator*(double a, const Dual<M>& b) {
  Dual<M> r;
  r.v = a * b.v;
#pragma unroll
  for (int m = 0; m < M; ++m) r.d[m] = a * b.d[m];
  return r;
}
// a / b as the IEEE quotient of the values; d(a/b) = (a' - (a/b) b') / b.
template <int M>
__device__ __forceinline__ Dual<M> operator/(const Dual<M>& a, const Dual<M>& b) {
  Dual<M> r;
  r.v = a.v / b.v;
  const double ib = 1.0 / b.v;
#pragma unroll
  for (int m = 0; m < M; ++m) r.d[m] = (a.d[m] - r.v * b.d[m]) * ib;
  return r;
}
template <int M>
__device__ __forceinline__ Dual<M> operator/(double a, const Dual<M>& b) {
  Dual<M> r;
  r.v = a / b.v;
  const double ib = 1.0 / b.v;
#pragma unroll
  for (int m = 0; m < M; ++m) r.d[m] = -r.v * b.d[m] * ib;
  return r;
}
template <int M>
__device__ __forceinline__ Dual<M> operator/(const Dual<M>& a, double b) {
  Dual<M> r;
  r.v = a.v / b;
#pragma unroll
  for (int m = 0; m < M; ++m) r.d[m] = a.d[m] / b;
  return r;
}

// fma with the value rounded once, as the double fma.
template <int M>
__device__ __forceinline__ Dual<M> fma(const Dual<M>& a, const Dual<M>& b, const Dual<M>& c) {
  Dual<M> r;
  r.v = ::fma(a.v, b.v, c.v);
#pragma unroll
  for (int m = 0; m < M; ++m) r.d[m] = ::fma(a.d[m], b.v, ::fma(a.v, b.d[m], c.d[m]));
  return r;
}
template <int M>
__device__ __forceinline__ Dual<M> fma(double a, const Dual<M>& b, const Dual<M>& c) {
  Dual<M> r;
  r.v = ::fma(a, b.v, c.v);
#pragma unroll
  for (int m = 0; m < M; ++m) r.d[m] = ::fma(a, b.d[m], c.d[m]);
  return r;
}
template <int M>
__device__ __forceinline__ Dual<M> fma(const Dual<M>& a, double b, const Dual<M>& c) {
  return fma(b, a, c);
}
template <int M>
__device__ __forceinline__ Dual<M> fma(const Dual<M>& a, const Dual<M>& b, double c) {
  Dual<M> r;
  r.v = ::fma(a.v, b.v, c);
#pragma unroll
  for (int m = 0; m < M; ++m) r.d[m] = ::fma(a.d[m], b.v, a.v * b.d[m]);
  return r;
}
template <int M>
__device__ __forceinline__ Dual<M> fma(double a, const Dual<M>& b, double c) {
  Dual<M> r;
  r.v = ::fma(a, b.v, c);
#pragma unroll
  for (int m = 0; m < M; ++m) r.d[m] = a * b.d[m];
  return r;
}
template <int M>
__device__ __forceinline__ Dual<M> fma(const Dual<M>& a, double b, double c) {
  return fma(b, a, c);
}

template <int M>
__device__ __forceinline__ Dual<M> exp(const Dual<M>& a) {
  Dual<M> r;
  r.v = ::exp(a.v);
#pragma unroll
  for (int m = 0; m < M; ++m) r.d[m] = r.v * a.d[m];
  return r;
}
template <int M>
__device__ __forceinline__ Dual<M> sqrt(const Dual<M>& a) {
  Dual<M> r;
  r.v = ::sqrt(a.v);
  const double h = 0.5 / r.v;
#pragma unroll
  for (int m = 0; m < M; ++m) r.d[m] = a.d[m] * h;
  return r;
}

}  // namespace ad
}  // namespace gs
