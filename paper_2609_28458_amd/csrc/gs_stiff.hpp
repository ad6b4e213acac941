// Device side of the stiff path: a Rosenbrock method, one trajectory per
// lane, for stiff systems (the paper's library pairs its explicit kernels
// with a Rosenbrock kernel, Sections "Adaptive explicit Runge-Kutta methods"
// and "Discussion"; it does not give the method).
//
// The method is Rodas4 (Hairer & Wanner 1996, Sec. IV.7; order 4, embedded
// order 3, stiffly accurate), in its transformed variables, which need no
// products with the Jacobian:
//   (1/(h gamma) I - J) u_i = f(y + sum_{j<i} a_ij u_j) + (1/h) sum_{j<i} c_ij u_j
//   y+ = y + sum_j m_j u_j,   error estimate e = u_s,   J = df/dy(y)
// for autonomous right-hand sides.  One LU factorisation with partial
// pivoting per attempt, six triangular solves.  Step control is the explicit
// path's (eq:errnorm, eq:controller with nu = 4); output times are landed on:
// a step that would pass the next output time is shortened to end there.
//
// Everything a lane needs lives in VGPRs: the matrix, the stages and the
// pivot indices are indexed only by compile-time constants (row swaps are
// per-lane branches over the candidate rows), so nothing goes to scratch.
// Reciprocals (of the pivots, h and h gamma, and the error scales) use the
// hardware reciprocal refined by Newton steps instead of IEEE division.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gs_kernels.hpp"

namespace gs {

// Rodas4 in transformed variables: gamma, a_ij, c_ij (below the diagonal),
// m_j.  The error weights are (0, ..., 0, 1).
struct Rodas4 {
  static constexpr int S = 6, ORDER = 4;
  static constexpr double GAMMA = 0.25;
  __host__ __device__ static constexpr double A(int i, int j) {
    constexpr double a[6][6] = {
        {0, 0, 0, 0, 0, 0},
        {1.544, 0, 0, 0, 0, 0},
        {0.9466785280815826, 0.2557011698983284, 0, 0, 0, 0},
        {3.314825187068521, 2.896124015972201, 0.9986419139977817, 0, 0, 0},
        {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 0, 0},
        {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 1.0, 0}};
    return a[i][j];
  }
  __host__ __device__ static constexpr double C(int i, int j) {
    constexpr double c[6][6] = {
        {0, 0, 0, 0, 0, 0},
        {-5.6688, 0, 0, 0, 0, 0},
        {-2.430093356833875, -0.2063599157091915, 0, 0, 0, 0},
        {-0.1073529058151375, -9.594562251023355, -20.47028614809616, 0, 0, 0},
        {7.496443313967647, -10.24680431464352, -33.99990352819905, 11.70890893206160, 0, 0},
        {8.083246795921522, -7.981132988064893, -31.52159432874371, 16.31930543123136,
         -6.058818238834054, 0}};
    return c[i][j];
  }
  __host__ __device__ static constexpr double M(int j) {
    constexpr double m[6] = {1.221224509226641, 6.019134481288629, 12.53708332932087,
                             -0.6878860361058950, 1.0, 1.0};
    return m[j];
  }
};

// ---------------------------------------------------------------------------
// Stiff mass-action kinetics (this library's own networks, with the same
// structure as the classic problems below).  f and the hand-written Jacobian.
//
// Kin3: y = (a, b, c), theta = (k1, k2, k3):
//   a -> b (k1 a),  b + c -> 2c (k2 b c),  c -> a (k3 c)
struct Kin3 {
  static constexpr int D = 3, P = 3;
  static constexpr int WAVES_PER_EU = 3;  // register budget of the stiff kernel
  template <class T>
  struct ParT {
    T k1, k2, k3;
  };
  using Par = ParT<double>;
  template <class T>
  __device__ static ParT<T> prep(const T (&th)[P]) {
    return ParT<T>{th[0], th[1], th[2]};
  }
  template <class T>
  __device__ static void f(double, const T (&y)[D], const ParT<T>& p, T (&dy)[D]) {
    const T r1 = p.k1 * y[0], r2 = p.k2 * y[1] * y[2], r3 = p.k3 * y[2];
    dy[0] = r3 - r1;
    dy[1] = r1 - r2;
    dy[2] = r2 - r3;
  }
  __device__ static void jac(const double (&y)[D], const Par& p, double (&J)[D][D]) {
    const double k2b = p.k2 * y[1], k2c = p.k2 * y[2];
    J[0][0] = -p.k1;
    J[0][1] = 0.0;
    J[0][2] = p.k3;
    J[1][0] = p.k1;
    J[1][1] = -k2c;
    J[1][2] = -k2b;
    J[2][0] = 0.0;
    J[2][1] = k2c;
    J[2][2] = k2b - p.k3;
  }
};

// Kin8: y1..y8, theta = (k1..k10, s, k12):
//   y1 <-> y2 (k1, k2), y2 -> y3 (k3), y3 <-> y4 (k4, k5),
//   y4 + y5 <-> y6 (k6, k7), y6 -> y7 (k8), y7 -> y8 (k9), y8 -> y1 (k10),
//   source -> y5 (s), y5 -> sink (k12)
struct Kin8 {
  static constexpr int D = 8, P = 12;
  static constexpr int WAVES_PER_EU = 1;
  template <class T>
  struct ParT {
    T k[P];
  };
  using Par = ParT<double>;
  template <class T>
  __device__ static ParT<T> prep(const T (&th)[P]) {
    ParT<T> p;
#pragma unroll
    for (int i = 0; i < P; ++i) p.k[i] = th[i];
    return p;
  }
  template <class T>
  __device__ static void f(double, const T (&y)[D], const ParT<T>& p, T (&dy)[D]) {
    const T r1 = p.k[0] * y[0], r2 = p.k[1] * y[1], r3 = p.k[2] * y[1], r4 = p.k[3] * y[2];
    const T r5 = p.k[4] * y[3], r6 = p.k[5] * y[3] * y[4], r7 = p.k[6] * y[5];
    const T r8 = p.k[7] * y[5], r9 = p.k[8] * y[6], r10 = p.k[9] * y[7];
    const T r12 = p.k[11] * y[4];
    dy[0] = r2 - r1 + r10;
    dy[1] = r1 - r2 - r3;
    dy[2] = r3 - r4 + r5;
    dy[3] = r4 - r5 - r6 + r7;
    dy[4] = r7 - r6 + p.k[10] - r12;
    dy[5] = r6 - r7 - r8;
    dy[6] = r8 - r9;
    dy[7] = r9 - r10;
  }
  __device__ static void jac(const double (&y)[D], const Par& p, double (&J)[D][D]) {
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int c = 0; c < D; ++c) J[r][c] = 0.0;
    const double k6y4 = p.k[5] * y[3], k6y5 = p.k[5] * y[4];
    J[0][0] = -p.k[0];
    J[0][1] = p.k[1];
    J[0][7] = p.k[9];
    J[1][0] = p.k[0];
    J[1][1] = -(p.k[1] + p.k[2]);
    J[2][1] = p.k[2];
    J[2][2] = -p.k[3];
    J[2][3] = p.k[4];
    J[3][2] = p.k[3];
    J[3][3] = -(p.k[4] + k6y5);
    J[3][4] = -k6y4;
    J[3][5] = p.k[6];
    J[4][3] = -k6y5;
    J[4][4] = -(k6y4 + p.k[11]);
    J[4][5] = p.k[6];
    J[5][3] = k6y5;
    J[5][4] = k6y4;
    J[5][5] = -(p.k[6] + p.k[7]);
    J[6][5] = p.k[7];
    J[6][6] = -p.k[8];
    J[7][6] = p.k[8];
    J[7][7] = -p.k[9];
  }
};

// ---------------------------------------------------------------------------
// The two classic stiff chemistry problems the paper names with its
// Rosenbrock kernel (Discussion: Robertson 1966; Schaefer 1975), in their
// standard form (Hairer & Wanner 1996, Sec. IV.1, IV.10) with the rate
// constants as per-trajectory parameters.
//
// Rober: y = (y1, y2, y3), theta = (k1, k2, k3), nominal (0.04, 3e7, 1e4):
//   y1' = -k1 y1 + k3 y2 y3,  y2' = k1 y1 - k3 y2 y3 - k2 y2^2,  y3' = k2 y2^2
struct Rober {
  static constexpr int D = 3, P = 3;
  static constexpr int WAVES_PER_EU = 3;
  template <class T>
  struct ParT {
    T k1, k2, k3;
  };
  using Par = ParT<double>;
  template <class T>
  __device__ static ParT<T> prep(const T (&th)[P]) {
    return ParT<T>{th[0], th[1], th[2]};
  }
  template <class T>
  __device__ static void f(double, const T (&y)[D], const ParT<T>& p, T (&dy)[D]) {
    const T r1 = p.k1 * y[0], r2 = p.k2 * y[1] * y[1], r3 = p.k3 * y[1] * y[2];
    dy[0] = r3 - r1;
    dy[1] = r1 - r3 - r2;
    dy[2] = r2;
  }
  __device__ static void jac(const double (&y)[D], const Par& p, double (&J)[D][D]) {
    const double k3y2 = p.k3 * y[1], k3y3 = p.k3 * y[2], k2y2 = 2.0 * p.k2 * y[1];
    J[0][0] = -p.k1;
    J[0][1] = k3y3;
    J[0][2] = k3y2;
    J[1][0] = p.k1;
    J[1][1] = -k3y3 - k2y2;
    J[1][2] = -k3y2;
    J[2][0] = 0.0;
    J[2][1] = k2y2;
    J[2][2] = 0.0;
  }
};

// Hires: y1..y8, theta = (a, b, c, s, d, e, kf, g), nominal (1.71, 0.43, 8.32,
// 0.0007, 0.035, 1.12, 280, 0.69); the problem's other constants are the sums
// 8.75 = c + b, 10.03 = c + a, 1.745 = a + d, 1.81 = e + g:
//   y1' = -a y1 + b y2 + c y3 + s        y5' = -(a + d) y5 + b y6 + b y7
//   y2' =  a y1 - (c + b) y2             y6' = -kf y6 y8 + g y4 + a y5 - b y6 + g y7
//   y3' = -(c + a) y3 + b y4 + d y5      y7' =  kf y6 y8 - (e + g) y7
//   y4' =  c y2 + a y3 - e y4            y8' = -kf y6 y8 + (e + g) y7
struct Hires {
  static constexpr int D = 8, P = 8;
  static constexpr int WAVES_PER_EU = 1;
  template <class T>
  struct ParT {
    T a, b, c, s, d, e, kf, g, cb, ca, ad, eg;
  };
  using Par = ParT<double>;
  template <class T>
  __device__ static ParT<T> prep(const T (&th)[P]) {
    ParT<T> p;
    p.a = th[0];
    p.b = th[1];
    p.c = th[2];
    p.s = th[3];
    p.d = th[4];
    p.e = th[5];
    p.kf = th[6];
    p.g = th[7];
    p.cb = p.c + p.b;
    p.ca = p.c + p.a;
    p.ad = p.a + p.d;
    p.eg = p.e + p.g;
    return p;
  }
  template <class T>
  __device__ static void f(double, const T (&y)[D], const ParT<T>& p, T (&dy)[D]) {
    const T r = p.kf * y[5] * y[7];
    dy[0] = -p.a * y[0] + p.b * y[1] + p.c * y[2] + p.s;
    dy[1] = p.a * y[0] - p.cb * y[1];
    dy[2] = -p.ca * y[2] + p.b * y[3] + p.d * y[4];
    dy[3] = p.c * y[1] + p.a * y[2] - p.e * y[3];
    dy[4] = -p.ad * y[4] + p.b * y[5] + p.b * y[6];
    dy[5] = -r + p.g * y[3] + p.a * y[4] - p.b * y[5] + p.g * y[6];
    dy[6] = r - p.eg * y[6];
    dy[7] = -r + p.eg * y[6];
  }
  __device__ static void jac(const double (&y)[D], const Par& p, double (&J)[D][D]) {
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int c = 0; c < D; ++c) J[r][c] = 0.0;
    const double ky8 = p.kf * y[7], ky6 = p.kf * y[5];
    J[0][0] = -p.a;
    J[0][1] = p.b;
    J[0][2] = p.c;
    J[1][0] = p.a;
    J[1][1] = -p.cb;
    J[2][2] = -p.ca;
    J[2][3] = p.b;
    J[2][4] = p.d;
    J[3][1] = p.c;
    J[3][2] = p.a;
    J[3][3] = -p.e;
    J[4][4] = -p.ad;
    J[4][5] = p.b;
    J[4][6] = p.b;
    J[5][3] = p.g;
    J[5][4] = p.a;
    J[5][5] = -ky8 - p.b;
    J[5][6] = p.g;
    J[5][7] = -ky6;
    J[6][5] = ky8;
    J[6][6] = -p.eg;
    J[6][7] = ky6;
    J[7][5] = -ky8;
    J[7][6] = p.eg;
    J[7][7] = -ky6;
  }
};

// ---------------------------------------------------------------------------
// LU factorisation with partial pivoting (the first row of largest |entry|
// in the column), in place: whole rows are swapped, multipliers stored below
// the diagonal, reciprocals of the pivots in inv.  False if a pivot is zero
// or not finite.
template <int D>
__device__ __forceinline__ bool lu_factor(double (&M)[D][D], int (&piv)[D], double (&inv)[D]) {
  bool ok = true;
  sfor<D>([&](auto K) {
    constexpr int k = decltype(K)::value;
    int p = k;
    double best = fabs(M[k][k]);
    sfor<D - k - 1>([&](auto R) {
      constexpr int r = k + 1 + decltype(R)::value;
      const double a = fabs(M[r][k]);
      p = a > best ? r : p;
      best = a > best ? a : best;
    });
    piv[k] = p;
    // The swap runs under a per-lane branch: a wavefront in which no lane
    // pivots at this column skips it.
    if (p != k) {
      sfor<D - k - 1>([&](auto R) {
        constexpr int r = k + 1 + decltype(R)::value;
        const bool sw = p == r;
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const double a = M[k][c], b = M[r][c];
          M[k][c] = sw ? b : a;
          M[r][c] = sw ? a : b;
        }
      });
    }
    ok = ok && best > 0.0 && (best - best) == 0.0;  // false for NaN and infinity
    inv[k] = fast_rcp(M[k][k]);
    sfor<D - k - 1>([&](auto R) {
      constexpr int r = k + 1 + decltype(R)::value;
      const double l = M[r][k] * inv[k];
      M[r][k] = l;
#pragma unroll
      for (int c = k + 1; c < D; ++c) M[r][c] = fma(-l, M[k][c], M[r][c]);
    });
  });
  return ok;
}

// x <- M^{-1} x with the factors of lu_factor; `swapped` says whether any
// row was exchanged (the permutation is skipped, per lane, when none was).
// Substitution runs column by column, so the updates of one step are
// independent of each other.
template <int D>
__device__ __forceinline__ void lu_solve(const double (&M)[D][D], const int (&piv)[D],
                                         const double (&inv)[D], bool swapped, double (&x)[D]) {
  if (swapped) {
    sfor<D>([&](auto K) {
      constexpr int k = decltype(K)::value;
      sfor<D - k - 1>([&](auto R) {
        constexpr int r = k + 1 + decltype(R)::value;
        const bool sw = piv[k] == r;
        const double a = x[k], b = x[r];
        x[k] = sw ? b : a;
        x[r] = sw ? a : b;
      });
    });
  }
#pragma unroll
  for (int c = 0; c < D - 1; ++c)
#pragma unroll
    for (int r = c + 1; r < D; ++r) x[r] = fma(-M[r][c], x[c], x[r]);
#pragma unroll
  for (int c = D - 1; c >= 0; --c) {
    x[c] *= inv[c];
#pragma unroll
    for (int r = 0; r < c; ++r) x[r] = fma(-M[r][c], x[c], x[r]);
  }
}

// One Rodas4 attempt of length h from y with f0 = f(y).  Returns the squared
// error norm (NaN if the matrix could not be factored) and y+ in yn.
template <class F>
__device__ __forceinline__ double rodas_attempt(const Inputs<F>& in, double t, double h,
                                                const double (&y)[F::D],
                                                const double (&f0)[F::D],
                                                double (&yn)[F::D]) {
  using TB = Rodas4;
  constexpr int D = F::D, S = TB::S;
  double M[D][D];
  F::jac(y, in.par, M);
  const double ig = fast_rcp(h * TB::GAMMA);
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) M[r][c] = (r == c ? ig : 0.0) - M[r][c];
  int piv[D];
  double inv[D];
  const bool ok = lu_factor<D>(M, piv, inv);
  bool swapped = false;
#pragma unroll
  for (int k = 0; k < D; ++k) swapped = swapped || piv[k] != k;
  const double ih = fast_rcp(h);
  double u[S][D];
  sfor<S>([&](auto I) {
    constexpr int i = decltype(I)::value;
    double x[D];
    if constexpr (i == 0) {
#pragma unroll
      for (int c = 0; c < D; ++c) x[c] = f0[c];
    } else {
      double Y[D];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        double acc = y[c], cu = 0.0;
        sfor<i>([&](auto J) {
          constexpr int j = decltype(J)::value;
          acc = fma(TB::A(i, j), u[j][c], acc);
          cu = fma(TB::C(i, j), u[j][c], cu);
        });
        Y[c] = acc;
        x[c] = cu;
      }
      double fy[D];
      F::f(t, Y, in.par, fy);
#pragma unroll
      for (int c = 0; c < D; ++c) x[c] = fma(ih, x[c], fy[c]);
    }
    lu_solve<D>(M, piv, inv, swapped, x);
#pragma unroll
    for (int c = 0; c < D; ++c) u[i][c] = x[c];
  });
  double sq = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    double acc = y[c];
    sfor<S>([&](auto J) {
      constexpr int j = decltype(J)::value;
      acc = fma(TB::M(j), u[j][c], acc);
    });
    yn[c] = acc;
    const double sc = fma(in.rtol, dmax(fabs(y[c]), fabs(acc)), in.atol);
    const double r = u[S - 1][c] * fast_rcp1(sc);
    sq = fma(r, r, sq);
  }
  const double en2 = sq * (1.0 / D);
  return ok ? en2 : __builtin_nan("");
}

// Persistent stiff solve, organised like the explicit forward kernel: an
// outer loop retires and refills lanes, an inner loop runs attempts of the
// live lanes until one of them finishes.  A wavefront refills once at least
// `refill` lanes are idle, with one atomic for all of them (a ballot and a
// prefix count in wave-uniform code), so the loads and the starting step of
// new trajectories are shared by many lanes instead of stalling the wave
// once per lane.  Static mode gives each lane one trajectory.
template <class F>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(F::WAVES_PER_EU)))
stiff_kernel(Params P) {
  using TB = Rodas4;
  constexpr int D = F::D;
  const int64_t n = P.n;
  const int lane = threadIdx.x & 63;
  int64_t idx = 0;
  bool live = false;
  bool queue_empty = P.sched_static != 0;  // wave-uniform
  Inputs<F> in;
  double y[D], f0[D];
  double t = 0.0, h = 0.0;
  double t_stop = 0.0;  // the next output time, or t1 after the last (in a register)
  int32_t nacc = 0, nrej = 0, nanrun = 0, kk = 0;

  auto store_node = [&](int q, const double (&v)[D]) {
#pragma unroll
    for (int c = 0; c < D; ++c) P.y_out[((int64_t)c * P.K + q) * n + idx] = v[c];
  };
  auto finish = [&](int32_t st) {
    for (int q = kk; q < P.K; ++q) {
#pragma unroll
      for (int c = 0; c < D; ++c) P.y_out[((int64_t)c * P.K + q) * n + idx] = __builtin_nan("");
    }
#pragma unroll
    for (int c = 0; c < D; ++c) P.y_final[(int64_t)c * n + idx] = y[c];
    P.n_acc[idx] = nacc;
    P.n_rej[idx] = nrej;
    P.status[idx] = st;
    live = false;
  };
  // Take trajectory i: load, validate, nodes at t0, first evaluation,
  // starting step.  Trajectories with nothing to integrate finish here.
  auto start = [&](int64_t i) {
    idx = i;
    live = true;
    nacc = nrej = nanrun = kk = 0;
    load_inputs<F>(P, i, in, y);
    t = in.t0;
    bool fin = true;
#pragma unroll
    for (int c = 0; c < D; ++c) fin = fin && (y[c] - y[c]) == 0.0;
    if (!inputs_valid<F>(P, i, in)) {
      finish(ST_BAD_INPUT);
      return;
    }
    while (kk < P.K && node_time(P, kk, i) <= in.t0) store_node(kk++, y);
    t_stop = kk < P.K ? node_time(P, kk, i) : in.t1;
    if (!fin) {
      finish(ST_NONFINITE);
      return;
    }
    if (!(in.t1 > in.t0)) {
      finish(ST_OK);
      return;
    }
    F::f(t, y, in.par, f0);
    h = P.h0 > 0.0 ? dmin(P.h0, in.t1 - in.t0) : initial_step<TB, F>(in, y, f0);
  };

  if (P.sched_static) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) start(g);
  }
  for (;;) {
    if (!queue_empty) {
      const uint64_t idle = __ballot(!live);
      const int nidle = __popcll(idle);
      if (nidle >= P.refill) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(P.counters, (unsigned long long)nidle);
        base = first_lane(base);
        if (base + (unsigned long long)nidle >= (unsigned long long)n) queue_empty = true;
        if (!live) {
          const unsigned long long pos = base + __popcll(idle & lanemask_lt());
          if (pos < (unsigned long long)n) {
            const int64_t id = P.order ? P.order[pos] : (int64_t)pos;
            if (id >= 0 && id < n) start(id);  // a bad permutation entry is skipped
          }
        }
      }
    }
    if (__ballot(live) == 0) {
      if (queue_empty) break;
      continue;
    }
    int32_t st = -1;  // status once this lane's trajectory has finished
    for (;;) {
      if (live) {
        if ((int64_t)nacc + nrej >= P.max_steps) {
          st = ST_MAX_STEPS;
        } else {
          const double stop = t_stop;
          double hh = h;
          bool land = false;
          if (t + hh >= stop) {
            hh = stop - t;
            land = true;
          }
          double yn[D];
          const double en2 = rodas_attempt<F>(in, t, hh, y, f0, yn);
          const bool finite = (en2 - en2) == 0.0;
          const double factor = step_factor<TB>(P, en2, 1.0, finite);
          bool done = false;
          if (finite && en2 <= 1.0) {
            ++nacc;
            t = land ? stop : t + hh;
            bool yfin = true;
#pragma unroll
            for (int c = 0; c < D; ++c) {
              y[c] = yn[c];
              yfin = yfin && (yn[c] - yn[c]) == 0.0;
            }
            if (!yfin) {
              st = ST_NONFINITE;
            } else {
              while (kk < P.K && t_stop <= t) {
                store_node(kk++, y);
                t_stop = kk < P.K ? node_time(P, kk, idx) : in.t1;
              }
              F::f(t, y, in.par, f0);
              nanrun = 0;
              done = t >= in.t1;
            }
          } else {
            ++nrej;
            nanrun = finite ? 0 : nanrun + 1;
            if (nanrun >= 50) st = ST_NONFINITE;
          }
          h = hh * factor;
          if (done)
            st = ST_OK;
          else if (st < 0 && underflow(h, t))
            st = ST_DT_UNDERFLOW;
        }
      }
      if (__ballot(live && st >= 0) != 0) break;
    }
    if (live && st >= 0) finish(st);
  }
}

// f of a stiff right-hand side at m points (SoA, point index fastest).
template <class F>
__global__ void __launch_bounds__(256) stiff_rhs_kernel(int64_t m, const double* y,
                                                        const double* theta, double* f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double yv[F::D], th[F::P], fv[F::D];
#pragma unroll
  for (int c = 0; c < F::D; ++c) yv[c] = y[(int64_t)c * m + i];
#pragma unroll
  for (int c = 0; c < F::P; ++c) th[c] = theta[(int64_t)c * m + i];
  F::f(0.0, yv, F::prep(th), fv);
#pragma unroll
  for (int c = 0; c < F::D; ++c) f[(int64_t)c * m + i] = fv[c];
}

}  // namespace gs
