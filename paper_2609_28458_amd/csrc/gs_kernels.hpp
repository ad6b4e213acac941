// Device side of the ensemble solver: one trajectory per wavefront lane.
//
// Every lane keeps its trajectory's state y, the stage derivatives k_j and
// the controller scalars in VGPRs; all loops over stages and components are
// unrolled at compile time so no array ever leaves registers.  The steps of
// the method follow the paper's Appendix "Numerical details":
//   stages and update          eq:rk
//   scaled RMS error norm      eq:errnorm
//   accept iff norm <= 1, new step from the (PI-generalised) controller
//                              eq:controller
//   outputs inside a step      eq:dense (polynomial), or a shortened step
//                              from the start of the step for Verner 7
// The derivative is the transpose of eq:stage-sens (reverse mode, steps held
// fixed), computed backwards over a tape that stores every accepted step or
// checkpoints from which segments are replayed (eq:cost).
//
// Wave-level votes (ballots) appear only where every lane of the wavefront
// executes them; values that steer a whole wave are made scalar with
// readfirstlane.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "gs_rhs.hpp"
#include "gs_tableaux.hpp"

namespace gs {

// ---------------------------------------------------------------------------
// Compile-time loops.
template <int I, int N, class Fn>
__device__ __forceinline__ void sfor_impl(Fn& fn) {
  if constexpr (I < N) {
    fn(std::integral_constant<int, I>{});
    sfor_impl<I + 1, N>(fn);
  }
}
template <int N, class Fn>
__device__ __forceinline__ void sfor(Fn&& fn) {
  sfor_impl<0, N>(fn);
}
// Descending: N-1, ..., 0.
template <int I, class Fn>
__device__ __forceinline__ void rfor_impl(Fn& fn) {
  if constexpr (I >= 0) {
    fn(std::integral_constant<int, I>{});
    rfor_impl<I - 1>(fn);
  }
}
template <int N, class Fn>
__device__ __forceinline__ void rfor(Fn&& fn) {
  rfor_impl<N - 1>(fn);
}

// std::min / std::max semantics (a NaN in the second argument is ignored the
// same way on every path).
__device__ __forceinline__ double dmin(double a, double b) { return (b < a) ? b : a; }
__device__ __forceinline__ double dmax(double a, double b) { return (a < b) ? b : a; }

// Every component of x (value and tangents) set to v.
__device__ __forceinline__ void set_all(double& x, double v) { x = v; }
template <int M>
__device__ __forceinline__ void set_all(ad::Dual<M>& x, double v) {
  x.v = v;
#pragma unroll
  for (int m = 0; m < M; ++m) x.d[m] = v;
}

// Zero of the solve's scalar type.
template <class T>
__device__ __forceinline__ T zero() {
  if constexpr (std::is_same<T, double>::value) {
    return 0.0;
  } else {
    return ad::constant<ad::width<T>::value>(0.0);
  }
}

constexpr int ST_OK = 0, ST_MAX_STEPS = 1, ST_DT_UNDERFLOW = 2, ST_NONFINITE = 3,
              ST_TAPE_OVERFLOW = 4, ST_BAD_INPUT = 5;

// Everything a kernel needs; a plain copy of the C-ABI arguments.
struct Params {
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
  double h0;
  double safety, amin, amax, beta1, beta2;
  int32_t ckpt_every;
  int32_t ckpt_cap;
  int32_t store;                // ckpt_every == 1: every accepted step is on the tape
  double* tape;                 // [slot][ckpt_cap][record], record as in tape_record
  int32_t* slot;                // [n]: tape slot of each trajectory (its queue position)
  unsigned long long* counters; // [0] forward queue, [1] adjoint queue, [2] replay mismatches
  const int64_t* order;
  int32_t refill;
  int32_t sched_static;
  int32_t fast_ctrl;  // I controller, default exponent, clamp bounds that hide the root's
                      // input clamp (decided on the host)
  int64_t n_wide;     // queue positions [0, n_wide) run 16 lanes per trajectory
  int32_t wide_blocks;  // the first wide_blocks workgroups run those
  int32_t out_layout;   // y_out: 0 = [d][K][n], 1 = [K][n][d]
  double* pending;      // [K][n][2 + d]: (start time, length, start state) of deferred
                        // shortened steps (pairs without a dense polynomial, K > 0)
};

struct VjpParams {
  int32_t R;           // losses handled by this launch (<= template R)
  int32_t r0;          // first loss index of this launch
  int32_t R_total;     // leading dimension of the cotangent arrays
  const double* ybar_out;
  const double* ybar_final;
  double* y0bar;
  double* thetabar;
  double* scratch;     // [lanes / 64][ckpt_every][2 + d][64], checkpoint mode only
  int32_t lds_bytes;   // host-side: dynamic LDS per block for the stage points
  double* adj;         // [lanes / 64][R][d + p][64], running cotangents of each lane
                       // (the launcher runs R = 1 per launch)
  int* occupancy_out;  // host-side, for the launcher's occupancy query only
};

__device__ __forceinline__ double node_time(const Params& P, int kk, int64_t i) {
  return P.t_out_stride ? P.t_out[(int64_t)kk * P.t_out_stride + i] : P.t_out[kk];
}
// Time of output node kk, or -infinity for kk < 0 (K >= 1): the load takes
// node 0 there and a select picks the result, so no branch guards the load.
__device__ __forceinline__ double node_time_or_ninf(const Params& P, int kk, int64_t i) {
  const double t = node_time(P, kk < 0 ? 0 : kk, i);
  return kk >= 0 ? t : -__builtin_inf();
}

// Per-trajectory inputs (theta and the constants derived from it in the
// scalar type of the solve: double, or ad::Dual for sensitivities).
template <class F, class T = double>
struct Inputs {
  T th[F::P];
  typename F::template ParT<T> par;
  double t0, t1, rtol, atol;
};

template <class F>
__device__ __forceinline__ void load_inputs(const Params& P, int64_t i, Inputs<F>& in,
                                            double (&y)[F::D]) {
#pragma unroll
  for (int c = 0; c < F::D; ++c) y[c] = P.y0[(int64_t)c * P.n + i];
#pragma unroll
  for (int c = 0; c < F::P; ++c)
    in.th[c] = P.theta_stride ? P.theta[(int64_t)c * P.theta_stride + i] : P.theta[c];
  in.par = F::prep(in.th);
  in.t0 = P.t0[P.t_stride ? i : 0];
  in.t1 = P.t1[P.t_stride ? i : 0];
  in.rtol = P.rtol[P.tol_stride ? i : 0];
  in.atol = P.atol[P.tol_stride ? i : 0];
}

// Checks that cannot be done on the host without reading device memory.
template <class F, class IN>
__device__ __forceinline__ bool inputs_valid(const Params& P, int64_t i, const IN& in) {
  bool ok = (in.t1 >= in.t0) && (in.rtol > 0.0) && (in.atol >= 0.0);
  double prev = in.t0;
  for (int kk = 0; kk < P.K; ++kk) {
    const double tk = node_time(P, kk, i);
    ok = ok && (tk >= prev) && (tk <= in.t1);
    prev = tk;
  }
  return ok;
}

// Starting step of Hairer, Norsett & Wanner (1993, Sec. II.4); the paper
// gives none.  RMS norms scaled by atol + rtol |y0|; one extra evaluation.
// Defined after inv_root; declared here for the kernels.
template <class TB, class F>
__device__ double initial_step(const Inputs<F>& in, const double (&y)[F::D],
                               const double (&f0)[F::D]);

// Stages 2..s of one step of length h from (t, y) with k[0] = f(t, y)
// given (eq:rk).  Returns y+ in yn.  For FSAL pairs the last stage point is
// y+ itself (its row of A is b), so yn costs nothing extra.
template <class TB, class F, class T>
__device__ __forceinline__ void rk_stages(const typename F::template ParT<T>& par, double t,
                                          double h, const T (&y)[F::D], T (&k)[TB::S][F::D],
                                          T (&yn)[F::D]) {
  constexpr int S = TB::S, D = F::D;
  sfor<S - 1>([&](auto J1) {
    constexpr int j = decltype(J1)::value + 1;
    T Y[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      T acc = zero<T>();
      sfor<j>([&](auto L) {
        constexpr int l = decltype(L)::value;
        constexpr double a = TB::A(j, l);
        if constexpr (a != 0.0) acc = fma(a, k[l][c], acc);
      });
      Y[c] = fma(h, acc, y[c]);
    }
    F::f(t + TB::C(j) * h, Y, par, k[j]);
    if constexpr (TB::FSAL && j == S - 1) {
#pragma unroll
      for (int c = 0; c < D; ++c) yn[c] = Y[c];
    }
  });
  if constexpr (!TB::FSAL) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      T acc = zero<T>();
      sfor<S>([&](auto J) {
        constexpr int j = decltype(J)::value;
        constexpr double b = TB::B(j);
        if constexpr (b != 0.0) acc = fma(b, k[j][c], acc);
      });
      yn[c] = fma(h, acc, y[c]);
    }
  }
}

// Square of the scaled RMS norm of eq:errnorm, for e = h sum_j (b_j -
// bhat_j) k_j.  The square suffices: accept iff it is <= 1, and the
// controller takes its power directly, so no square root is needed.
template <class TB, class F, class T>
__device__ __forceinline__ double error_norm2(double h, const T (&y)[F::D], const T (&yn)[F::D],
                                              const T (&k)[TB::S][F::D], double rtol,
                                              double atol) {
  constexpr int D = F::D;
  double sq[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    double e = 0.0;
    sfor<TB::S>([&](auto J) {
      constexpr int j = decltype(J)::value;
      constexpr double w = TB::E(j);
      if constexpr (w != 0.0) e = fma(w, ad::val(k[j][c]), e);
    });
    e *= h;
    const double sc = fma(rtol, dmax(fabs(ad::val(y[c])), fabs(ad::val(yn[c]))), atol);
    const double r = e * fast_rcp1(sc);
    sq[c] = r * r;
  }
  // pairwise sum: a shorter dependency chain at the end of the attempt
#pragma unroll
  for (int w = 1; w < D; w *= 2) {
#pragma unroll
    for (int c = 0; c + w < D; c += 2 * w) sq[c] += sq[c + w];
  }
  return sq[0] * (1.0 / D);
}

// r^M by repeated squaring (M a compile-time constant).
template <int M>
__device__ __forceinline__ double ipow(double r) {
  if constexpr (M == 1) {
    return r;
  } else if constexpr (M % 2 == 0) {
    const double h = ipow<M / 2>(r);
    return h * h;
  } else {
    return ipow<M - 1>(r) * r;
  }
}

// x^(-1/M) for x in [1e-30, 1e30]: an FP32 seed from the hardware log2/exp2,
// then two Newton steps on r^M x = 1 in FP64 (relative error ~(M+1)/2 eps^2
// per step, so full double precision after two).  A single third-order
// correction reaches the same error bound with fewer dependent operations,
// but lands on a different last bit than the oracle's pow more often; the
// step sizes then drift apart at the rounding level and the 900-step
// precession solves leave the 1e-9 parity bar, so the Newton steps stay.
template <int M>
__device__ __forceinline__ double inv_root(double x) {
  const float lx = __builtin_amdgcn_logf(static_cast<float>(x));
  double r = static_cast<double>(__builtin_amdgcn_exp2f(lx * (-1.0f / M)));
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double u = ipow<M>(r) * x;
    r = fma(r * (1.0 / M), 1.0 - u, r);
  }
  return r;
}

template <class TB, class F>
__device__ double initial_step(const Inputs<F>& in, const double (&y)[F::D],
                               const double (&f0)[F::D]) {
  constexpr int D = F::D;
  const double span = in.t1 - in.t0;
  double isc[D];
  double d0 = 0.0, d1 = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    isc[c] = fast_rcp(in.atol + fabs(y[c]) * in.rtol);
    d0 = fma(y[c] * isc[c], y[c] * isc[c], d0);
    d1 = fma(f0[c] * isc[c], f0[c] * isc[c], d1);
  }
  d0 = sqrt(d0 * (1.0 / D));
  d1 = sqrt(d1 * (1.0 / D));
  double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 * fast_rcp(d1);
  h0 = dmin(h0, span);
  double y1[D], f1[D];
#pragma unroll
  for (int c = 0; c < D; ++c) y1[c] = y[c] + h0 * f0[c];
  F::f(in.t0 + h0, y1, in.par, f1);
  double d2 = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double r = (f1[c] - f0[c]) * isc[c];
    d2 = fma(r, r, d2);
  }
  d2 = sqrt(d2 * (1.0 / D)) * fast_rcp(h0);
  double h1;
  if (d1 <= 1e-15 && d2 <= 1e-15) {
    h1 = dmax(1e-6, h0 * 1e-3);
  } else {
    // (0.01 / max(d1, d2))^(1/nu)
    const double x = dmax(d1, d2) * 100.0;
    h1 = (x >= 1e-30 && x <= 1e30) ? inv_root<TB::ORDER>(x) : pow(x, -1.0 / TB::ORDER);
  }
  return dmin(dmin(100.0 * h0, h1), span);
}

// Value at t + sigma h inside an accepted step, evaluated once the step is
// committed.  Polynomial pairs use eq:dense rewritten about the end of the
// step, y + h sum_j b_j(sigma) k_j = y+ - h sum_j (b_j - b_j(sigma)) k_j, so the
// start state need not stay live; Verner 7 takes a shortened step of length
// sigma h from (t, y_start) reusing k[0] = f(t, y_start).  The shortened
// step runs in the step's own stage array: it overwrites k[1..s-1] (which a
// pair without FSAL no longer needs once the step is accepted: its next
// first stage is evaluated afresh) and keeps k[0], so several outputs in one
// step each start from the same k[0].  A second stage array for it would
// double the lane's largest live set.
template <class TB, class F, class T>
__device__ __forceinline__ void dense_value(const typename F::template ParT<T>& par, double t,
                                            double h, double sigma, const T (&y_end)[F::D],
                                            const T (&y_start)[F::D], T (&k)[TB::S][F::D],
                                            T (&out)[F::D]) {
  constexpr int S = TB::S, D = F::D;
  if constexpr (TB::POLY_DENSE) {
    double w[S];
    sfor<S>([&](auto J) {
      constexpr int j = decltype(J)::value;
      double acc = 0.0;
      rfor<TB::DEG>([&](auto Q) {
        constexpr int q = decltype(Q)::value;
        acc = fma(acc, sigma, TB::Bs(j, q));
      });
      w[j] = TB::B(j) - acc * sigma;
    });
#pragma unroll
    for (int c = 0; c < D; ++c) {
      T acc = zero<T>();
#pragma unroll
      for (int j = 0; j < S; ++j) acc = fma(w[j], k[j][c], acc);
      out[c] = fma(-h, acc, y_end[c]);
    }
  } else {
    static_assert(!TB::FSAL, "shortened-step outputs reuse the stages of a pair without FSAL");
    rk_stages<TB, F>(par, t, sigma * h, y_start, k, out);
  }
}

// Controller of eq:controller from the squared norm en2 = ||e||^2.  The
// paper's I form safety * ||e||^(-1/nu) = safety * en2^(-1/(2 nu)) takes the
// Newton root (P.fast_ctrl, decided once per launch so the branch is
// uniform).  Clamping en2 to [1e-30, 1e30] changes nothing: the host sets
// fast_ctrl only when safety * 1e15^(1/nu) >= alpha_max and
// safety * 1e-15^(1/nu) <= alpha_min, so outside that range the raw factor
// would be clamped to the same bound anyway.  The PI
// form (beta2 != 0) or another exponent uses pow; the previous norm is kept
// squared (err_prev2 = max(||e_prev||^2, 1e-8), i.e. ||e_prev|| floored at
// 1e-4) so no square root is taken on the hot path.
template <class TB>
__device__ __forceinline__ double step_factor(const Params& P, double en2, double err_prev2,
                                              bool finite) {
  double raw;
  if (P.fast_ctrl) {
    const double x = dmin(dmax(en2, 1e-30), 1e30);
    raw = P.safety * inv_root<2 * TB::ORDER>(x);
  } else {
    const double b1 = P.beta1 > 0.0 ? P.beta1 : 1.0 / TB::ORDER;
    raw = P.safety * pow(en2, -0.5 * b1);
    if (P.beta2 != 0.0) raw *= pow(err_prev2, 0.5 * P.beta2);
  }
  raw = (en2 == 0.0) ? P.amax : raw;
  raw = finite ? raw : P.amin;
  return dmin(P.amax, dmax(P.amin, raw));
}

__device__ __forceinline__ bool underflow(double h, double t) {
  return fabs(h) < 16.0 * 2.220446049250313e-16 * dmax(fabs(t), 1.0);
}

// Integration state of one lane.
template <class TB, class F, class T = double>
struct Traj {
  static constexpr int S = TB::S, D = F::D;
  Inputs<F, T> in;
  T y[D];
  T k[S][D];
  double t, h;
  double err_prev2;  // squared norm of the last accepted step (PI control)
  int32_t nacc, nrej, nanrun;
  int32_t ck_left;   // accepted steps until the next checkpoint
};

// Outcome of one attempt.
struct Attempt {
  bool accepted;
  bool finished;
  int32_t status;
  double t_start, h_used, t_new;
};

// One step attempt with everything the controller does after it.  The
// accept/reject update is written as per-lane selects (no divergent
// branch around the state); only output nodes run under a branch:
// `on_accept(s, t_start, h, y_start)` sees y = y+, t = t_new and the step's
// stages k (k[0] still f(t_start, y_start)); y_start is only meaningful for
// shortened-step pairs, whose outputs may overwrite k[1..s-1] (see
// dense_value).
template <class TB, class F, class T, class OnAccept>
__device__ __forceinline__ Attempt attempt(const Params& P, Traj<TB, F, T>& s,
                                           OnAccept&& on_accept) {
  constexpr int S = TB::S, D = F::D;
  Attempt a;
  a.t_start = s.t;
  bool last = false;
  double hh = s.h;
  if (s.t + hh >= s.in.t1) {
    hh = s.in.t1 - s.t;
    last = true;
  }
  a.h_used = hh;
  T yn[D];
  rk_stages<TB, F>(s.in.par, s.t, hh, s.y, s.k, yn);
  const double en2 = error_norm2<TB, F>(hh, s.y, yn, s.k, s.in.rtol, s.in.atol);
  // x - x == 0 exactly when x is finite; no short-circuit branches.
  const bool finite = (en2 - en2) == 0.0;
  const double factor = step_factor<TB>(P, en2, s.err_prev2, finite);
  const bool acc = finite & (en2 <= 1.0);
  a.accepted = acc;
  const double t_new = last ? s.in.t1 : s.t + hh;
  a.t_new = t_new;
  // The step's start state goes to on_accept where an output may need it:
  // a shortened step, or a deferred output (plain solves).  A dual-number
  // solve of a polynomial pair needs only the end state.
  constexpr bool KEEP_START = !TB::POLY_DENSE || std::is_same<T, double>::value;
  T ystart[D];
  double probe = 0.0;  // becomes NaN if any component of y+ is not finite
#pragma unroll
  for (int c = 0; c < D; ++c) {
    if constexpr (KEEP_START) ystart[c] = s.y[c];
    probe = fma(ad::val(yn[c]), 0.0, probe);
    s.y[c] = ad::select(acc, yn[c], s.y[c]);
  }
  const bool fin = probe == 0.0;
  s.t = acc ? t_new : s.t;
  if (acc) {
    if constexpr (KEEP_START) {
      on_accept(s, a.t_start, hh, ystart);
    } else {
      on_accept(s, a.t_start, hh, s.y);
    }
  }
  if constexpr (TB::FSAL && !std::is_same<T, double>::value) {
    // For dual numbers the first stage is copied under the accept branch:
    // a select between the two stage arrays placed after that branch was
    // turned into a choice between their addresses, which kept the lane's
    // whole state in scratch memory.
    if (acc) {
#pragma unroll
      for (int c = 0; c < D; ++c) s.k[0][c] = s.k[S - 1][c];
    }
  } else if constexpr (TB::FSAL) {
#pragma unroll
    for (int c = 0; c < D; ++c) s.k[0][c] = ad::select(acc, s.k[S - 1][c], s.k[0][c]);
  } else {
    // A rejected lane recomputes f at its unchanged (t, y): the same value.
    F::f(s.t, s.y, s.in.par, s.k[0]);
  }
  s.err_prev2 = acc ? dmax(en2, 1e-8) : s.err_prev2;
  s.nacc += acc ? 1 : 0;
  s.nrej += acc ? 0 : 1;
  s.nanrun = finite ? 0 : s.nanrun + 1;
  s.h = hh * factor;
  const bool bad_state = acc & !fin;
  const bool nan_fail = !finite & (s.nanrun >= 50);
  const bool done = acc & last;
  const bool tiny = !done & underflow(s.h, s.t);
  a.finished = bad_state | nan_fail | done | tiny;
  a.status = (bad_state | nan_fail) ? ST_NONFINITE : (tiny ? ST_DT_UNDERFLOW : ST_OK);
  return a;
}

// Tape records of trajectory i.  Checkpoint mode (ckpt_every >= 2): record c
// holds (t, h, err_prev2, y, f(t, y)) after c * ckpt_every accepted steps, all
// a replay needs to restart the controller.  Store mode (ckpt_every == 1):
// record n holds (t_n, h_{n-1}, y_n) for n = 0..N, the start of every
// accepted step and the length of the step that led to it, so the adjoint
// and dense queries need no replay.
template <class F>
__host__ __device__ constexpr int ckpt_record_len() { return 3 + 2 * F::D; }
template <class F>
__host__ __device__ constexpr int store_record_len() { return 2 + F::D; }

// A trajectory's records sit in the tape slot of the queue position the
// forward took it from (slot[i]), not at its index: the lanes of a wave take
// neighbouring positions, so their records are neighbours in memory and the
// translation of their addresses stays within few pages, where a caller's
// order (longest first) would scatter them over the whole tape.
template <class TB, class F>
__device__ __forceinline__ double* tape_record(const Params& P, int64_t slot, int c) {
  const int rec = P.store ? store_record_len<F>() : ckpt_record_len<F>();
  return P.tape + ((int64_t)slot * P.ckpt_cap + c) * rec;
}

template <class TB, class F>
__device__ __forceinline__ void write_store_record(const Params& P, int64_t slot, int n, double t,
                                                   double h_in, const double (&y)[F::D]) {
  double* r = P.tape + ((int64_t)slot * P.ckpt_cap + n) * store_record_len<F>();
  r[0] = t;
  r[1] = h_in;
#pragma unroll
  for (int j = 0; j < F::D; ++j) r[2 + j] = y[j];
}

template <class TB, class F>
__device__ __forceinline__ void write_checkpoint(const Params& P, int64_t slot, int c,
                                                 const Traj<TB, F>& s) {
  double* r = tape_record<TB, F>(P, slot, c);
  r[0] = s.t;
  r[1] = s.h;
  r[2] = s.err_prev2;
#pragma unroll
  for (int j = 0; j < F::D; ++j) {
    r[3 + j] = s.y[j];
    r[3 + F::D + j] = s.k[0][j];
  }
}

template <class TB, class F>
__device__ __forceinline__ void read_checkpoint(const Params& P, int64_t slot, int c,
                                                Traj<TB, F>& s) {
  const double* r = tape_record<TB, F>(P, slot, c);
  s.t = r[0];
  s.h = r[1];
  s.err_prev2 = r[2];
#pragma unroll
  for (int j = 0; j < F::D; ++j) {
    s.y[j] = r[3 + j];
    s.k[0][j] = r[3 + F::D + j];
  }
  s.nanrun = 0;
}

// Lane 0's value in every lane, as a scalar the compiler knows is uniform,
// so branches on it are uniform (no ballot ever sits in a divergent region).
__device__ __forceinline__ unsigned long long first_lane(unsigned long long x) {
  const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(x));
  const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(x >> 32));
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// ---------------------------------------------------------------------------
// Forward solve.  Persistent grid: each lane holds one trajectory; when at
// least `refill` lanes of a wavefront are idle, one atomic fetches that many
// queue positions and the idle lanes take them (ballot + prefix count).  In
// static mode lane g integrates trajectory g and is never refilled.
// Occupancy target of the forward kernel: the stage array k[S][D] dominates
// the live registers; up to 63 doubles (126 VGPRs) two waves per SIMD fit in
// the 512-entry register file without spilling, beyond that one.
#ifndef GS_FWD_WAVES
#define GS_FWD_WAVES 2
#endif
template <class TB, class F>
struct FwdOccupancy {
  static constexpr int waves = (TB::S * F::D > 63) ? 1 : GS_FWD_WAVES;
};


// Sensitivity columns of a forward-mode solve (eq:sens, eq:stage-sens):
// column m seeds the initial-condition component col[m] (< d) or the
// parameter col[m] - d; tangents of every output land in S_final
// [d][M][n] and S_out [d][M][K][n].  Step control reads values only, so the
// steps are those of the plain solve.
struct SensParams {
  int32_t col[4];      // this launch's columns (template M of them)
  int32_t m_total;     // columns of the output arrays
  int32_t m0;          // first output column of this launch
  double* S_final;
  double* S_out;
  int* occupancy_out;  // host-side, for the launcher's occupancy query only
};

// Seeded dual inputs: column m is the derivative with respect to
// y0[col[m]] (col[m] < d) or theta[col[m] - d]; par is prepared from the
// seeded theta so it carries d par / d theta.
template <class F, int M>
__device__ __forceinline__ void seed_inputs(const SensParams& SP, const Inputs<F>& ind,
                                            const double (&y0)[F::D], Inputs<F, ad::Dual<M>>& in,
                                            ad::Dual<M> (&y)[F::D]) {
#pragma unroll
  for (int c = 0; c < F::D; ++c) {
    y[c].v = y0[c];
#pragma unroll
    for (int m = 0; m < M; ++m) y[c].d[m] = SP.col[m] == c ? 1.0 : 0.0;
  }
#pragma unroll
  for (int q = 0; q < F::P; ++q) {
    in.th[q].v = ind.th[q];
#pragma unroll
    for (int m = 0; m < M; ++m) in.th[q].d[m] = SP.col[m] == F::D + q ? 1.0 : 0.0;
  }
  in.par = F::prep(in.th);
  in.t0 = ind.t0;
  in.t1 = ind.t1;
  in.rtol = ind.rtol;
  in.atol = ind.atol;
}

// ---------------------------------------------------------------------------
// Group mode: one trajectory on a group of 16 lanes (a DPP row), lane c of
// the group holding component c of the state and of every stage.  Stage
// sums and error terms are the single-lane expressions for that component;
// the right-hand side is evaluated per component where one is written for
// the row (RowRhs), else each stage point is broadcast within the row so
// that every lane evaluates the ordinary right-hand side on the full vector
// and keeps its component; the norm sums the broadcast terms of lanes
// 0..d-1 in the pairwise order of error_norm2.  A group therefore takes the
// same steps, bit for bit, as a single lane, with about a sixth of the stage
// arithmetic on the critical path of one trajectory.
constexpr int kGroup = 16;

// A DPP move of a double within each row of 16 lanes.  Lanes whose source
// lies outside the row read 0 (bound_ctrl); no old value is kept, so no
// register is cleared first.  Callers run it with every lane of the row
// active (DPP is convergent: the compiler keeps it out of divergent code).
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
// Lane SRC of this lane's row, in every lane of the row (row_newbcast, the
// one DPP control that moves 64 bits in one instruction on this chip).
template <int SRC>
__device__ __forceinline__ double row_bcast(double v) {
  return __longlong_as_double(
      __builtin_amdgcn_mov_dpp(__double_as_longlong(v), 0x150 + SRC, 0xF, 0xF, true));
}
// The same for a dual number: the value and each tangent.
template <int SRC, int M>
__device__ __forceinline__ ad::Dual<M> row_bcast(const ad::Dual<M>& v) {
  ad::Dual<M> r;
  r.v = row_bcast<SRC>(v.v);
#pragma unroll
  for (int m = 0; m < M; ++m) r.d[m] = row_bcast<SRC>(v.d[m]);
  return r;
}
// Sum of lanes 0..D-1 of the row, in every lane of the row: each value is
// broadcast and the sum taken in the pairwise order of error_norm2 (pairs,
// then pairs of pairs, ...), so a group's norm has the bits of one lane's.
template <int D>
__device__ __forceinline__ double row_sum(double v) {
  double q[D];
  sfor<D>([&](auto C) {
    constexpr int c = decltype(C)::value;
    q[c] = row_bcast<c>(v);
  });
#pragma unroll
  for (int w = 1; w < D; w *= 2) {
#pragma unroll
    for (int c = 0; c + w < D; c += 2 * w) q[c] += q[c + w];
  }
  return q[0];
}

// Full vector of the row's components (lanes 0..D-1), in every lane.
template <int D, class T>
__device__ __forceinline__ void row_gather(const T& v, T (&out)[D]) {
  sfor<D>([&](auto C) {
    constexpr int c = decltype(C)::value;
    out[c] = row_bcast<c>(v);
  });
}
// Component c of a full vector (c is the lane's own index).  Written as
// bit masks: as a chain of selects the compiler turns it into a store of
// the vector to scratch and an indexed load.
template <int D>
__device__ __forceinline__ double pick(const double (&v)[D], int c) {
  unsigned long long r = __double_as_longlong(v[0]);
#pragma unroll
  for (int j = 1; j < D; ++j) {
    const unsigned long long m = 0ull - (unsigned long long)(c == j);
    r = (r & ~m) | ((unsigned long long)__double_as_longlong(v[j]) & m);
  }
  return __longlong_as_double((long long)r);
}
template <int D, int M>
__device__ __forceinline__ ad::Dual<M> pick(const ad::Dual<M> (&v)[D], int c) {
  double part[D];
  ad::Dual<M> r;
#pragma unroll
  for (int j = 0; j < D; ++j) part[j] = v[j].v;
  r.v = pick<D>(part, c);
#pragma unroll
  for (int m = 0; m < M; ++m) {
#pragma unroll
    for (int j = 0; j < D; ++j) part[j] = v[j].d[m];
    r.d[m] = pick<D>(part, c);
  }
  return r;
}

// Component c of f(t, Y) for the row whose lane c holds Y[c]: the full
// vector is gathered, every lane evaluates the right-hand side and keeps its
// component; lanes c >= D get 0.
template <class F>
struct RowRhs {
  __device__ static double f(double t, double yc, const typename F::Par& p, int c) {
    double Y[F::D], kf[F::D];
    row_gather<F::D>(yc, Y);
    F::f(t, Y, p, kf);
    return c < F::D ? pick<F::D>(kf, c) : 0.0;
  }
};

// The logarithmic halo (eq:loghalo) written per component: the positions
// are broadcast for the denominator, lane c < 3 takes the velocity from lane
// c + 3 (row_shl:3) and lane 3 <= c < 6 its position from lane c - 3
// (row_shr:3), times the lane's weight (1, 1, 1/q^2 for c = 3, 4, 5; 0
// beyond, so lanes c >= 6 get 0 while the state is finite).  The weight
// depends only on the lane and the parameters, so the compiler keeps it out
// of the attempt loop.  Every expression and its order are those of
// LogHalo::f (1 * x is exact), so the result is bit-identical to component
// c of the full evaluation.
template <>
struct RowRhs<LogHalo> {
  __device__ static double f(double, double yc, const LogHalo::Par& p, int c) {
    const double x = row_bcast<0>(yc), y = row_bcast<1>(yc), z = row_bcast<2>(yc);
    const double vel = dpp_mov<0x103>(yc);
    const double pos = dpp_mov<0x113>(yc);
    const double Dn = fma(z * z, p.iq2, fma(y, y, fma(x, x, p.rc2)));
    const double s = -p.v02 * fast_rcp(Dn);
    const double w = c == 5 ? p.iq2 : (c < 6 ? 1.0 : 0.0);
    return c < 3 ? vel : s * (w * pos);
  }
};

// Component c of f for the solve's scalar type: the per-component form of
// the row for double, and for dual numbers (sensitivity solves) the gathered
// vector through the ordinary right-hand side, which is exactly the
// arithmetic of one lane's sensitivity solve.
template <class F, class T>
__device__ __forceinline__ T row_f(double t, const T& yc,
                                   const typename F::template ParT<T>& p, int c) {
  if constexpr (std::is_same<T, double>::value) {
    return RowRhs<F>::f(t, yc, p, c);
  } else {
    T Y[F::D], kf[F::D];
    row_gather<F::D>(yc, Y);
    F::f(t, Y, p, kf);
    return c < F::D ? pick<F::D>(kf, c) : zero<T>();
  }
}

// The tableau's coefficients in vector registers for the group loop.  As
// immediates every 64-bit coefficient costs two scalar moves per use inside
// the loop (the compiler rematerialises them rather than keep 60+ scalar
// registers), and each scalar move takes an issue slot of the wavefront on
// the critical path.  Passing each value once through an empty asm statement
// with a VGPR constraint hides that it is a constant, so it is loaded before
// the loop and stays in a VGPR; the values, and so the results, are the
// tableau's own.  Entries that the tableau has as zero are never read.
template <class TB>
struct GroupCoef {
  double a[TB::S][TB::S], b[TB::S], e[TB::S], c[TB::S];
  __device__ __forceinline__ void load() {
    sfor<TB::S>([&](auto J) {
      constexpr int j = decltype(J)::value;
      sfor<TB::S>([&](auto L) {
        constexpr int l = decltype(L)::value;
        if constexpr (l < j && TB::A(j, l) != 0.0) a[j][l] = hold(TB::A(j, l));
      });
      if constexpr (TB::B(j) != 0.0) b[j] = hold(TB::B(j));
      if constexpr (TB::E(j) != 0.0) e[j] = hold(TB::E(j));
      if constexpr (TB::C(j) != 0.0) c[j] = hold(TB::C(j));
    });
  }
  // Node j of the stage times (0 where the tableau has 0).
  template <int j>
  __device__ __forceinline__ double node() const {
    if constexpr (TB::C(j) != 0.0) {
      return c[j];
    } else {
      return 0.0;
    }
  }
  __device__ static __forceinline__ double hold(double v) {
    asm("" : "+v"(v));
    return v;
  }
};

template <class TB, class F, class T = double>
struct GroupTraj {
  static constexpr int S = TB::S, D = F::D;
  Inputs<F, T> in;
  T y;     // own component (0 beyond d)
  T k[S];  // own component of each stage derivative
  double t, h, err_prev2;
  int32_t nacc, nrej, nanrun;
  int32_t ck_left;  // accepted steps until the next checkpoint
};

// One attempt of a group: the single-lane attempt() component by component
// (for a dual scalar type the error estimate and step control read the
// values only, as one lane's do).  on_accept(t_old, h, y_old) runs on
// acceptance with the new state in s and the step's stages still in s.k, as
// in the single-lane attempt.
template <class TB, class F, class T, class OnAccept>
__device__ __forceinline__ Attempt group_attempt(const Params& P, const GroupCoef<TB>& cf,
                                                 GroupTraj<TB, F, T>& s, int c,
                                                 OnAccept&& on_accept) {
  constexpr int S = TB::S, D = F::D;
  Attempt a;
  a.t_start = s.t;
  bool last = false;
  double hh = s.h;
  if (s.t + hh >= s.in.t1) {
    hh = s.in.t1 - s.t;
    last = true;
  }
  a.h_used = hh;
  T yn = zero<T>();
  // The sums over stages in push form: as soon as k_l is known its terms
  // enter the partial sums of every later stage, of the update and of the
  // error estimate.  Each sum still takes its terms in ascending l, as the
  // single-lane attempt does, so the values are the same bit for bit; what
  // changes is that only a_{j,j-1} k_{j-1} and the step stand between one
  // stage's right-hand side and the next stage point, and the other terms
  // fill the latency of the evaluation in flight.
  T accs[S], accb = zero<T>();
  double e = 0.0;  // the error estimate reads values only
#pragma unroll
  for (int j = 0; j < S; ++j) accs[j] = zero<T>();
  auto push = [&](auto L) {
    constexpr int l = decltype(L)::value;
    sfor<S>([&](auto J) {
      constexpr int j = decltype(J)::value;
      if constexpr (j > l && TB::A(j, l) != 0.0) accs[j] = fma(cf.a[j][l], s.k[l], accs[j]);
    });
    if constexpr (!TB::FSAL && TB::B(l) != 0.0) accb = fma(cf.b[l], s.k[l], accb);
    if constexpr (TB::E(l) != 0.0) e = fma(cf.e[l], ad::val(s.k[l]), e);
  };
  push(std::integral_constant<int, 0>{});
  sfor<S - 1>([&](auto J1) {
    constexpr int j = decltype(J1)::value + 1;
    const T Yc = fma(hh, accs[j], s.y);
    s.k[j] = row_f<F>(s.t + cf.template node<j>() * hh, Yc, s.in.par, c);
    if constexpr (TB::FSAL && j == S - 1) yn = Yc;
    push(std::integral_constant<int, j>{});
  });
  if constexpr (!TB::FSAL) yn = fma(hh, accb, s.y);
  e *= hh;
  const double sc = fma(s.in.rtol, dmax(fabs(ad::val(s.y)), fabs(ad::val(yn))), s.in.atol);
  const double r = e * fast_rcp1(sc);
  const double en2 = row_sum<D>(r * r) * (1.0 / D);
  const bool finite = (en2 - en2) == 0.0;
  const double factor = step_factor<TB>(P, en2, s.err_prev2, finite);
  const bool acc = finite & (en2 <= 1.0);
  a.accepted = acc;
  const double t_new = last ? s.in.t1 : s.t + hh;
  a.t_new = t_new;
  const bool fin = row_sum<D>(fma(ad::val(yn), 0.0, 0.0)) == 0.0;
  const T y_old = s.y;
  s.y = ad::select(acc, yn, s.y);
  s.t = acc ? t_new : s.t;
  if (acc) on_accept(a.t_start, hh, y_old);
  if constexpr (TB::FSAL) {
    s.k[0] = ad::select(acc, s.k[S - 1], s.k[0]);
  } else {
    s.k[0] = row_f<F>(s.t, s.y, s.in.par, c);
  }
  s.err_prev2 = acc ? dmax(en2, 1e-8) : s.err_prev2;
  s.nacc += acc ? 1 : 0;
  s.nrej += acc ? 0 : 1;
  s.nanrun = finite ? 0 : s.nanrun + 1;
  s.h = hh * factor;
  const bool bad_state = acc & !fin;
  const bool nan_fail = !finite & (s.nanrun >= 50);
  const bool done = acc & last;
  const bool tiny = !done & underflow(s.h, s.t);
  a.finished = bad_state | nan_fail | done | tiny;
  a.status = (bad_state | nan_fail) ? ST_NONFINITE : (tiny ? ST_DT_UNDERFLOW : ST_OK);
  return a;
}

// Component of the dense output (eq:dense) of a pair with a dense
// polynomial, for the group lane that holds this component: the expression
// and order of dense_value, so the value is that of one lane.
template <class TB, class T>
__device__ __forceinline__ T group_dense(double h, double sigma, const T& y_end,
                                         const T (&k)[TB::S]) {
  constexpr int S = TB::S;
  double w[S];
  sfor<S>([&](auto J) {
    constexpr int j = decltype(J)::value;
    double acc = 0.0;
    rfor<TB::DEG>([&](auto Q) {
      constexpr int q = decltype(Q)::value;
      acc = fma(acc, sigma, TB::Bs(j, q));
    });
    w[j] = TB::B(j) - acc * sigma;
  });
  T acc = zero<T>();
#pragma unroll
  for (int j = 0; j < S; ++j) acc = fma(w[j], k[j], acc);
  return fma(-h, acc, y_end);
}

// Component of a shortened-step output (a pair without a dense
// polynomial): the step of length hs from (t, y_start) with k[0] =
// f(t, y_start), as rk_stages takes it for one lane (sums from zero in
// ascending l, the tableau's own nodes), so the value is that of one lane.
// Overwrites k[1..s-1], which an accepted step of a pair without FSAL no
// longer needs.
template <class TB, class F, class T>
__device__ __forceinline__ T group_short_step(const typename F::template ParT<T>& par,
                                              double t, double hs, const T& y_start,
                                              T (&k)[TB::S], int c) {
  constexpr int S = TB::S;
  static_assert(!TB::FSAL, "shortened-step outputs reuse the stages of a pair without FSAL");
  sfor<S - 1>([&](auto J1) {
    constexpr int j = decltype(J1)::value + 1;
    T acc = zero<T>();
    sfor<j>([&](auto L) {
      constexpr int l = decltype(L)::value;
      constexpr double a = TB::A(j, l);
      if constexpr (a != 0.0) acc = fma(a, k[l], acc);
    });
    k[j] = row_f<F>(t + TB::C(j) * hs, fma(hs, acc, y_start), par, c);
  });
  T acc = zero<T>();
  sfor<S>([&](auto J) {
    constexpr int j = decltype(J)::value;
    constexpr double b = TB::B(j);
    if constexpr (b != 0.0) acc = fma(b, k[j], acc);
  });
  return fma(hs, acc, y_start);
}

// The group part of a forward launch: workgroups [0, wide_blocks) take the
// queue positions [0, n_wide) (the head of the order, longest first when
// the caller sorts by predicted cost), one per 16-lane group, from their own
// queue head (counters[3]).  Control mirrors the single-lane loop; every
// ballot sits where all lanes of the wave execute it.  TAPE: the tape in
// store mode (every accepted step) or checkpoint mode (every ckpt_every
// accepted steps), written as one lane writes it: lane c of the group
// stores component c of each record (and of k1 in a checkpoint), lane 0 its
// time, step and controller memory.
// NODES: output nodes, written as one lane writes them (lane c component c):
// exact hits directly, the others as deferred records (lane 0 the step's
// start time and length, lane c component c of its start state), or with
// INLOOP (a pair with a dense polynomial, no pending array) the dense value.
// T = ad::Dual<M>: a sensitivity solve (no tape), lane c carrying component
// c of the value and its M tangents; outputs are evaluated in the loop (the
// dense value, or Verner 7's shortened step on the group) and the tangents
// land in S_out and S_final as one lane writes them.
template <class TB, class F, class T, bool NODES, bool TAPE, bool INLOOP>
__device__ void solve_group(const Params& P, const SensParams& SP) {
  constexpr int D = F::D;
  constexpr bool SENS = !std::is_same<T, double>::value;
  constexpr int M = ad::width<T>::value;
  static_assert(!(SENS && TAPE), "sensitivity solves keep no tape");
  constexpr bool DEFER = NODES && !INLOOP && !SENS;
  const int lane = threadIdx.x & 63;
  const int c = lane & (kGroup - 1);
  const int first = lane & ~(kGroup - 1);  // the group's lane 0
  GroupTraj<TB, F, T> s;
  GroupCoef<TB> cf;
  cf.load();
  int64_t idx = -1, ts = 0;  // trajectory and its tape slot
  bool live = false, overflow = false;
  bool queue_empty = false;
  int kp = 0;                           // next output node
  double t_next = __builtin_inf();      // its time, kept in a register

  auto put_node = [&](int kk, const T& v, double t_start = 0.0, double hs = 0.0) {
    if constexpr (DEFER) {
      double* rec = P.pending + ((int64_t)kk * P.n + idx) * (2 + D);
      if (c == 0) rec[1] = hs;
      if (hs != 0.0) {
        if (c == 0) rec[0] = t_start;
        if (c < D) rec[2 + c] = ad::val(v);
        return;
      }
    }
    if (c < D) {
      P.y_out[P.out_layout ? ((int64_t)kk * P.n + idx) * D + c
                           : ((int64_t)c * P.K + kk) * P.n + idx] = ad::val(v);
      if constexpr (SENS) {
#pragma unroll
        for (int m = 0; m < M; ++m)
          SP.S_out[(((int64_t)c * SP.m_total + SP.m0 + m) * P.K + kk) * P.n + idx] = v.d[m];
      }
    }
  };
  auto put_record = [&](int n, double h_in) {
    double* r = P.tape + ((int64_t)ts * P.ckpt_cap + n) * store_record_len<F>();
    if (c < D) r[2 + c] = ad::val(s.y);
    if (c == 0) {
      r[0] = s.t;
      r[1] = h_in;
    }
  };
  auto put_checkpoint = [&](int cidx) {
    double* r = P.tape + ((int64_t)ts * P.ckpt_cap + cidx) * ckpt_record_len<F>();
    if (c == 0) {
      r[0] = s.t;
      r[1] = s.h;
      r[2] = s.err_prev2;
    }
    if (c < D) {
      r[3 + c] = ad::val(s.y);
      r[3 + D + c] = ad::val(s.k[0]);
    }
  };
  auto finish = [&](int32_t st) {
    if constexpr (NODES) {
      T nan_v = zero<T>();
      set_all(nan_v, __builtin_nan(""));
      for (; kp < P.K; ++kp) put_node(kp, nan_v);
    }
    if (c < D) {
      P.y_final[(int64_t)c * P.n + idx] = ad::val(s.y);
      if constexpr (SENS) {
#pragma unroll
        for (int m = 0; m < M; ++m)
          SP.S_final[((int64_t)c * SP.m_total + SP.m0 + m) * P.n + idx] = s.y.d[m];
      }
    }
    if (c == 0) {
      P.n_acc[idx] = s.nacc;
      P.n_rej[idx] = s.nrej;
      P.status[idx] = (st == ST_OK && overflow) ? ST_TAPE_OVERFLOW : st;
    }
    live = false;
  };
  auto start = [&](int64_t i, int64_t slot) {
    idx = i;
    ts = slot;
    live = true;
    overflow = false;
    if constexpr (TAPE) {
      if (c == 0) P.slot[i] = (int32_t)slot;
    }
    s.nacc = s.nrej = s.nanrun = 0;
    s.err_prev2 = 1.0;
    Inputs<F> ind;  // the double inputs (the starting-step rule reads values)
    double y0[D];
    load_inputs<F>(P, i, ind, y0);
    T yv[D];  // the initial state, seeded for a sensitivity solve
    if constexpr (SENS) {
      seed_inputs<F, M>(SP, ind, y0, s.in, yv);
    } else {
      s.in = ind;
#pragma unroll
      for (int j = 0; j < D; ++j) yv[j] = y0[j];
    }
    s.t = s.in.t0;
    s.y = c < D ? pick<D>(yv, c) : zero<T>();
    bool fin = true;
#pragma unroll
    for (int j = 0; j < D; ++j) fin = fin && (y0[j] == y0[j]) && (fabs(y0[j]) < __builtin_inf());
    kp = 0;
    if (!inputs_valid<F>(P, i, s.in)) {
      finish(ST_BAD_INPUT);
      return;
    }
    // Nodes at t0 take y0.
    while (NODES && kp < P.K && node_time(P, kp, i) <= s.in.t0) {
      put_node(kp, s.y);
      ++kp;
    }
    if constexpr (NODES) t_next = kp < P.K ? node_time(P, kp, i) : __builtin_inf();
    if (!fin) {
      finish(ST_NONFINITE);
      return;
    }
    if (!(s.in.t1 > s.in.t0)) {
      finish(ST_OK);
      return;
    }
    T f0[D];
    double f0v[D];
    F::f(s.t, yv, s.in.par, f0);
#pragma unroll
    for (int j = 0; j < D; ++j) f0v[j] = ad::val(f0[j]);
    s.k[0] = c < D ? pick<D>(f0, c) : zero<T>();
    s.h = P.h0 > 0.0 ? dmin(P.h0, s.in.t1 - s.in.t0) : initial_step<TB, F>(ind, y0, f0v);
    s.ck_left = P.ckpt_every;
    if constexpr (TAPE) {
      if (P.ckpt_cap <= 0)
        overflow = true;
      else if (P.store)
        put_record(0, 0.0);
      else
        put_checkpoint(0);
    }
  };

  for (;;) {
    if (!queue_empty) {
      // one bit per idle group (its lane 0)
      const uint64_t idle = __ballot(!live && c == 0);
      const int nidle = __popcll(idle);
      if (nidle > 0) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(P.counters + 3, (unsigned long long)nidle);
        base = first_lane(base);
        if (base + (unsigned long long)nidle >= (unsigned long long)P.n_wide) queue_empty = true;
        if (!live) {
          const uint64_t below = first ? (~0ull >> (64 - first)) : 0ull;
          const unsigned long long pos = base + __popcll(idle & below);
          if (pos < (unsigned long long)P.n_wide) {
            const int64_t id = P.order ? P.order[pos] : (int64_t)pos;
            if (id >= 0 && id < P.n) start(id, (int64_t)pos);
          }
        }
      }
    }
    if (__ballot(live) == 0) {
      if (queue_empty) break;
      continue;
    }
    int32_t st = -1;
    for (;;) {
      if (live) {
        if ((int64_t)s.nacc + s.nrej >= P.max_steps) {
          st = ST_MAX_STEPS;
        } else {
          const Attempt a = group_attempt<TB, F>(
              P, cf, s, c, [&](double t_old, double hh, const T& y_old) {
                if constexpr (!NODES) return;
                while (t_next <= s.t) {
                  const double tq = t_next;
                  if (tq == s.t) {
                    put_node(kp, s.y);
                  } else if constexpr (DEFER) {
                    put_node(kp, y_old, t_old,
                             TB::POLY_DENSE ? hh : ((tq - t_old) / hh) * hh);
                  } else if constexpr (TB::POLY_DENSE) {
                    put_node(kp, group_dense<TB>(hh, (tq - t_old) / hh, s.y, s.k));
                  } else {
                    put_node(kp, group_short_step<TB, F>(s.in.par, t_old,
                                                         ((tq - t_old) / hh) * hh, y_old, s.k, c));
                  }
                  ++kp;
                  t_next = kp < P.K ? node_time(P, kp, idx) : __builtin_inf();
                }
              });
          if constexpr (!TAPE) {
          } else if (P.store) {
            // every accepted step, the last one included
            if (a.accepted) {
              if (s.nacc < P.ckpt_cap)
                put_record(s.nacc, a.h_used);
              else
                overflow = true;
            }
          } else if (!a.finished) {
            s.ck_left -= a.accepted ? 1 : 0;
            if (s.ck_left == 0) {
              s.ck_left = P.ckpt_every;
              const int cidx = s.nacc / P.ckpt_every;
              if (cidx < P.ckpt_cap)
                put_checkpoint(cidx);
              else
                overflow = true;
            }
          }
          if (a.finished) st = a.status;
        }
      }
      if (__ballot(live && st >= 0) != 0) break;
    }
    if (live && st >= 0) finish(st);
  }
}

// NODES: the call has output nodes (K > 0); TAPE: it keeps a checkpoint
// tape.  The host picks the variant, so a plain solve runs a loop with
// neither check in it.
// The forward solve for scalar type T (double, or ad::Dual<M> carrying M
// sensitivity columns).  Persistent grid: each lane holds one trajectory;
// when at least `refill` lanes of a wavefront are idle, one atomic fetches
// that many queue positions and the idle lanes take them (ballot + prefix
// count).  In static mode lane g integrates trajectory g and is never
// refilled.
template <class TB, class F, class T, bool NODES, bool TAPE, bool INLOOP = false>
__device__ __forceinline__ void forward_body(const Params& P, const SensParams& SP) {
  constexpr int D = F::D;
  constexpr bool SENS = !std::is_same<T, double>::value;
  constexpr int M = ad::width<T>::value;
  static_assert(!(SENS && TAPE), "sensitivity solves keep no tape");
  // The plain solve defers outputs inside a step to short_step_kernel (one
  // thread per output, after the solve): it records the step's start time,
  // length and start state, and the later kernel takes the step again (a
  // pair with a dense polynomial) or the shortened step (a pair without).
  // In the attempt loop an output then costs a few stores instead of the
  // dense evaluation, which a wavefront otherwise runs with most lanes idle
  // on nearly every attempt once outputs are dense.  The host supplies the
  // pending array; where it has no room for it (INLOOP, a pair with a dense
  // polynomial only) the outputs are evaluated in the loop, as they are for
  // sensitivity solves.
  static_assert(!INLOOP || TB::POLY_DENSE, "in-loop outputs need a dense polynomial");
  constexpr bool DEFER = NODES && !SENS && !INLOOP;
  Traj<TB, F, T> s;
  int64_t idx = -1, ts = 0;  // trajectory and its tape slot
  int32_t kp = 0;
  double t_next = 0.0;  // time of output node kp, kept in a register (infinity after the last)
  bool live = false, overflow = false;
  bool queue_empty = P.sched_static != 0;  // wave-uniform
  const int lane = threadIdx.x & 63;

  // Output node kk of the lane's trajectory: values, and tangents.  A
  // deferred shortened step (hs > 0) is recorded instead, (t_start, hs,
  // y_start) in one contiguous record of pending [K][n][2 + d]; a value
  // written now marks its record done (hs = 0).
  auto put_node = [&](int kk, const T (&v)[D], double t_start = 0.0, double hs = 0.0) {
    if constexpr (DEFER) {
      double* rec = P.pending + ((int64_t)kk * P.n + idx) * (2 + D);
      rec[1] = hs;
      if (hs != 0.0) {
        rec[0] = t_start;
#pragma unroll
        for (int c = 0; c < D; ++c) rec[2 + c] = ad::val(v[c]);
        return;
      }
    }
#pragma unroll
    for (int c = 0; c < D; ++c) {
      P.y_out[P.out_layout ? ((int64_t)kk * P.n + idx) * D + c
                           : ((int64_t)c * P.K + kk) * P.n + idx] = ad::val(v[c]);
      if constexpr (SENS) {
#pragma unroll
        for (int m = 0; m < M; ++m)
          SP.S_out[(((int64_t)c * SP.m_total + SP.m0 + m) * P.K + kk) * P.n + idx] = v[c].d[m];
      }
    }
  };
  // Write the final results of the lane's trajectory and free the lane.
  auto finish = [&](int32_t st) {
    for (; NODES && kp < P.K; ++kp) {
      T nan_v[D];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        nan_v[c] = zero<T>();
        set_all(nan_v[c], __builtin_nan(""));
      }
      put_node(kp, nan_v);
    }
#pragma unroll
    for (int c = 0; c < D; ++c) {
      P.y_final[(int64_t)c * P.n + idx] = ad::val(s.y[c]);
      if constexpr (SENS) {
#pragma unroll
        for (int m = 0; m < M; ++m)
          SP.S_final[((int64_t)c * SP.m_total + SP.m0 + m) * P.n + idx] = s.y[c].d[m];
      }
    }
    P.n_acc[idx] = s.nacc;
    P.n_rej[idx] = s.nrej;
    P.status[idx] = (st == ST_OK && overflow) ? ST_TAPE_OVERFLOW : st;
    live = false;
  };

  // Take trajectory i at tape slot `slot`: load, validate, first
  // evaluation, starting step.
  auto start = [&](int64_t i, int64_t slot) {
    idx = i;
    ts = slot;
    if constexpr (TAPE) P.slot[i] = (int32_t)slot;
    live = true;
    kp = 0;
    overflow = false;
    s.nacc = s.nrej = s.nanrun = 0;
    s.err_prev2 = 1.0;
    Inputs<F> ind;  // the double inputs (the starting-step rule reads values)
    double y0[D];
    load_inputs<F>(P, i, ind, y0);
    if constexpr (SENS) {
      seed_inputs<F, M>(SP, ind, y0, s.in, s.y);
    } else {
      s.in = ind;
#pragma unroll
      for (int c = 0; c < D; ++c) s.y[c] = y0[c];
    }
    s.t = s.in.t0;
    bool fin = true;
#pragma unroll
    for (int c = 0; c < D; ++c) fin = fin && (y0[c] == y0[c]) && (fabs(y0[c]) < __builtin_inf());
    if (!inputs_valid<F>(P, i, s.in)) {
      finish(ST_BAD_INPUT);
      return;
    }
    // Nodes at t0 take y0.
    while (NODES && kp < P.K && node_time(P, kp, i) <= s.in.t0) {
      put_node(kp, s.y);
      ++kp;
    }
    if constexpr (NODES) t_next = kp < P.K ? node_time(P, kp, i) : __builtin_inf();
    if (!fin) {
      finish(ST_NONFINITE);
      return;
    }
    if (!(s.in.t1 > s.in.t0)) {
      finish(ST_OK);
      return;
    }
    F::f(s.t, s.y, s.in.par, s.k[0]);
    if (P.h0 > 0.0) {
      s.h = dmin(P.h0, s.in.t1 - s.in.t0);
    } else {
      double f0[D];
#pragma unroll
      for (int c = 0; c < D; ++c) f0[c] = ad::val(s.k[0][c]);
      s.h = initial_step<TB, F>(ind, y0, f0);
    }
    s.ck_left = P.ckpt_every;
    if constexpr (TAPE) {
      if (P.ckpt_cap <= 0)
        overflow = true;
      else if (P.store)
        write_store_record<TB, F>(P, ts, 0, s.t, 0.0, s.y);
      else
        write_checkpoint<TB, F>(P, ts, 0, s);
    }
  };

  if (P.sched_static) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < P.n) start(g, g);
  }

  // Outer loop: bookkeeping (retire, refill).  Inner loop: step attempts of
  // the live lanes until one of them finishes, so the hot loop holds only
  // the attempt and the rare output and checkpoint writes.
  for (;;) {
    if (!queue_empty) {
      const uint64_t idle = __ballot(!live);
      const int nidle = __popcll(idle);
      if (nidle >= P.refill) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(P.counters, (unsigned long long)nidle);
        base = first_lane(base);
        if (base + (unsigned long long)nidle >= (unsigned long long)P.n) queue_empty = true;
        if (!live) {
          const unsigned long long pos = base + __popcll(idle & lanemask_lt());
          if (pos < (unsigned long long)P.n) {
            const int64_t id = P.order ? P.order[pos] : (int64_t)pos;
            if (id >= 0 && id < P.n) start(id, (int64_t)pos);  // a bad entry is skipped
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
        if ((int64_t)s.nacc + s.nrej >= P.max_steps) {
          st = ST_MAX_STEPS;
        } else {
          const Attempt a = attempt<TB, F>(
              P, s, [&](Traj<TB, F, T>& sa, double t_old, double hh, const T (&ys)[D]) {
                if constexpr (!NODES) return;
                // the next output time sits in a register: memory is read only
                // when an output is passed, not on every accepted step
                while (t_next <= sa.t) {
                  const double tq = t_next;
                  if (tq == sa.t) {
                    put_node(kp, sa.y);
                  } else if constexpr (DEFER) {
                    // the step from (t_old, ys) is taken again later, in
                    // short_step_kernel; here its start and length (the
                    // shortened length for a pair without a polynomial)
                    put_node(kp, ys, t_old, TB::POLY_DENSE ? hh : ((tq - t_old) / hh) * hh);
                  } else {
                    T out[D];
                    dense_value<TB, F>(sa.in.par, t_old, hh, (tq - t_old) / hh, sa.y, ys, sa.k,
                                       out);
                    put_node(kp, out);
                  }
                  ++kp;
                  t_next = kp < P.K ? node_time(P, kp, idx) : __builtin_inf();
                }
              });
          if constexpr (!TAPE) {
          } else if (P.store) {
            // Every accepted step, the last one included.
            if (a.accepted) {
              if (s.nacc < P.ckpt_cap)
                write_store_record<TB, F>(P, ts, s.nacc, s.t, a.h_used, s.y);
              else
                overflow = true;
            }
          } else if (!a.finished) {
            s.ck_left -= a.accepted ? 1 : 0;
            if (s.ck_left == 0) {
              s.ck_left = P.ckpt_every;
              const int c = s.nacc / P.ckpt_every;
              if (c < P.ckpt_cap)
                write_checkpoint<TB, F>(P, ts, c, s);
              else
                overflow = true;
            }
          }
          if (a.finished) st = a.status;
        }
      }
      if (__ballot(live && st >= 0) != 0) break;
    }
    if (live && st >= 0) finish(st);
  }
}


// Plain forward solve (and, with wide > 0, the head of the queue on 16-lane
// groups).
// INLOOP: outputs of a pair with a dense polynomial evaluated in the loop
// (no pending array).
template <class TB, class F, bool NODES, bool TAPE, bool INLOOP = false>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(FwdOccupancy<TB, F>::waves, 8))) solve_kernel(Params P) {
  if constexpr (F::D <= kGroup) {
    if ((int)blockIdx.x < P.wide_blocks) {  // uniform per workgroup
      solve_group<TB, F, double, NODES, TAPE, INLOOP>(P, SensParams{});
      return;
    }
  }
  forward_body<TB, F, double, NODES, TAPE, INLOOP>(P, SensParams{});
}

// The deferred outputs of a plain solve: for output kk of trajectory i the
// solve recorded in pending the start (t_start, y_start) and a length hs.
// A pair with a dense polynomial takes the step of length hs again and
// evaluates the polynomial of eq:dense at the output's sigma; a pair without
// one takes the shortened step of length hs.  k[0] = f(t_start, y_start) is
// evaluated afresh: for a first-same-as-last pair it is the value the solve
// carried over from the previous step (the same function at the same time
// and state), so every output equals the one the solve would have written,
// bit for bit.  One thread per output, over [K][n] (consecutive threads
// write consecutive trajectories of y_out); hs = 0 marks an output the solve
// already wrote.
template <class TB, class F>
__global__ void __launch_bounds__(256) short_step_kernel(Params P) {
  constexpr int D = F::D;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)P.K * P.n) return;
  const int64_t i = g % P.n;
  const int64_t kk = g / P.n;
  const double* rec = P.pending + g * (2 + D);
  const double hs = rec[1];
  if (hs == 0.0) return;
  const double t_start = rec[0];
  Inputs<F> in;
  double y0_unused[D];
  load_inputs<F>(P, i, in, y0_unused);
  double y[D], k[TB::S][D], out[D];
#pragma unroll
  for (int c = 0; c < D; ++c) y[c] = rec[2 + c];
  F::f(t_start, y, in.par, k[0]);
  if constexpr (TB::POLY_DENSE) {
    double yend[D];
    rk_stages<TB, F>(in.par, t_start, hs, y, k, yend);
    const double tq = node_time(P, (int)kk, i);
    dense_value<TB, F>(in.par, t_start, hs, (tq - t_start) / hs, yend, y, k, out);
  } else {
    rk_stages<TB, F>(in.par, t_start, hs, y, k, out);
  }
#pragma unroll
  for (int c = 0; c < D; ++c)
    P.y_out[P.out_layout ? (kk * P.n + i) * D + c : ((int64_t)c * P.K + kk) * P.n + i] = out[c];
}

// Forward solve with M sensitivity columns in the same launch.  WIDE: the
// launch runs the head of the order on 16-lane groups (a variant of its own,
// so that a launch without groups keeps the single-lane register budget).
template <class TB, class F, int M, bool NODES, bool WIDE>
__global__ void __launch_bounds__(256) sens_kernel(Params P, SensParams SP) {
  if constexpr (WIDE && F::D <= kGroup) {
    if ((int)blockIdx.x < P.wide_blocks) {  // uniform per workgroup
      solve_group<TB, F, ad::Dual<M>, NODES, false, false>(P, SP);
      return;
    }
  }
  forward_body<TB, F, ad::Dual<M>, NODES, false>(P, SP);
}

// ---------------------------------------------------------------------------
// A stage can receive a cotangent only through y+ (b_j != 0), a later stage
// (a_ij != 0) or a dense output; this decides it at compile time for the
// first two routes.
template <class TB>
__host__ __device__ constexpr bool stage_feeds_step(int j) {
  if (TB::B(j) != 0.0) return true;
  for (int i = j + 1; i < TB::S; ++i)
    if (TB::A(i, j) != 0.0) return true;
  return false;
}
// The first stage of the reverse sweep that adds to stage l's cotangent (the
// last feeding stage i > l with a_il != 0), or -1 if none does.
template <class TB>
__host__ __device__ constexpr int first_touch(int l) {
  for (int i = TB::S - 1; i > l; --i)
    if (stage_feeds_step<TB>(i) && TB::A(i, l) != 0.0) return i;
  return -1;
}

// Reverse of one explicit RK step of length h from (t, y) (the transpose of
// eq:stage-sens with h fixed).  lam[r] enters as the cotangent of y+ and
// leaves as the cotangent of y; thb[r] accumulates the parameter cotangent.
// seed(r, kb, yb) adds the cotangents of outputs inside the step: for a
// polynomial dense pair an output at sigma with cotangent g adds
// h b_j(sigma) g to stage j and g to y.  all_stages also reverses the stages
// that only the dense output reads.
//
// The stage points Y_1 .. Y_{s-1} are recomputed first and kept until the
// reverse sweep reads them: in registers when there are few of them and no
// output cotangents enter (vjp_stages_in_lds false: (s - 1) d <= 36 and no
// output nodes, as in the orbit-gradient workload), else parked in the
// lane's slice of LDS (ysc, stride `ys` between values, so the lanes of a
// workgroup touch consecutive words), which keeps only the stage cotangents
// in registers and the stage points off HBM.  In registers they cost no LDS
// traffic, which the four waves of a fully loaded CU otherwise share; with
// output nodes (whose seeds add a runtime loop and the dense-only stages)
// the register form measured wrong cotangents in one variant at the
// register limit (Tsit5 on the dark-energy system), so those keep LDS.
template <class TB, class F, bool NODES>
__host__ __device__ constexpr bool vjp_stages_in_lds() {
  return NODES || (TB::S - 1) * F::D > 36;
}

template <class TB, class F, int R, bool NODES, class Seed>
__device__ __forceinline__ void reverse_step(const Inputs<F>& in, double t, double h,
                                             const double (&y)[F::D], double (&lam)[R][F::D],
                                             double (&thb)[R][F::P], bool all_stages,
                                             Seed&& seed, double* ysc, int ys) {
  constexpr int S = TB::S, D = F::D;
  constexpr bool LDS = vjp_stages_in_lds<TB, F, NODES>();
  // Every slot is defined on every path: a stage that only the dense output
  // reads is written and read under the same runtime flag, and a slot left
  // unwritten on one path must not reach the register allocator as undefined.
  double Yr[LDS ? 1 : S - 1][D];
  if constexpr (!LDS) {
#pragma unroll
    for (int j = 0; j < S - 1; ++j)
#pragma unroll
      for (int c = 0; c < D; ++c) Yr[j][c] = 0.0;
  }
  auto Ys = [&](int j, int c) -> double& {
    if constexpr (LDS) {
      return ysc[((j - 1) * D + c) * ys];
    } else {
      return Yr[j - 1][c];
    }
  };
  {
    double k[S][D];
    F::f(t, y, in.par, k[0]);
    sfor<S - 1>([&](auto J1) {
      constexpr int j = decltype(J1)::value + 1;
      if (stage_feeds_step<TB>(j) || (TB::POLY_DENSE && all_stages)) {
        double Yj[D];
#pragma unroll
        for (int c = 0; c < D; ++c) {
          double acc = 0.0;
          sfor<j>([&](auto L) {
            constexpr int l = decltype(L)::value;
            constexpr double a = TB::A(j, l);
            if constexpr (a != 0.0) acc = fma(a, k[l][c], acc);
          });
          Yj[c] = fma(h, acc, y[c]);
          Ys(j, c) = Yj[c];
        }
        if constexpr (j < S - 1) F::f(t + TB::C(j) * h, Yj, in.par, k[j]);
      }
    });
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if constexpr (!NODES) {
      // No output seeds: stage j's cotangent (h b_j lam plus what later
      // stages add) is formed when it is first added to, so that only the
      // accumulators of stages still ahead in the sweep are live (seven of
      // ten for Verner 7 instead of all).  Same operations in the same order
      // as the form below.
      double kb[S][D];
      double yb[D];
#pragma unroll
      for (int c = 0; c < D; ++c) yb[c] = lam[r][c];
      rfor<S>([&](auto J) {
        constexpr int j = decltype(J)::value;
        if constexpr (stage_feeds_step<TB>(j)) {
          double Yj[D], ybj[D], kbj[D];
          if constexpr (j == 0) {
#pragma unroll
            for (int c = 0; c < D; ++c) Yj[c] = y[c];
          } else {
#pragma unroll
            for (int c = 0; c < D; ++c) Yj[c] = Ys(j, c);
          }
#pragma unroll
          for (int c = 0; c < D; ++c) {
            if constexpr (first_touch<TB>(j) >= 0)
              kbj[c] = kb[j][c];
            else
              kbj[c] = (h * TB::B(j)) * lam[r][c];
          }
          F::vjp(t + TB::C(j) * h, Yj, in.th, in.par, kbj, ybj, thb[r]);
#pragma unroll
          for (int c = 0; c < D; ++c) yb[c] += ybj[c];
          sfor<j>([&](auto L) {
            constexpr int l = decltype(L)::value;
            constexpr double a = TB::A(j, l);
            if constexpr (a != 0.0) {
#pragma unroll
              for (int c = 0; c < D; ++c) {
                if constexpr (first_touch<TB>(l) == j)
                  kb[l][c] = fma(h * a, ybj[c], (h * TB::B(l)) * lam[r][c]);
                else
                  kb[l][c] = fma(h * a, ybj[c], kb[l][c]);
              }
            }
          });
        }
      });
#pragma unroll
      for (int c = 0; c < D; ++c) lam[r][c] = yb[c];
      continue;
    }
    double kb[S][D];
    double yb[D];
    sfor<S>([&](auto J) {
      constexpr int j = decltype(J)::value;
      constexpr double b = TB::B(j);
#pragma unroll
      for (int c = 0; c < D; ++c) kb[j][c] = (h * b) * lam[r][c];
    });
#pragma unroll
    for (int c = 0; c < D; ++c) yb[c] = lam[r][c];
    seed(r, kb, yb);
    rfor<S>([&](auto J) {
      constexpr int j = decltype(J)::value;
      if (stage_feeds_step<TB>(j) || (TB::POLY_DENSE && all_stages)) {
        double Yj[D], ybj[D];
        if constexpr (j == 0) {
#pragma unroll
          for (int c = 0; c < D; ++c) Yj[c] = y[c];
        } else {
#pragma unroll
          for (int c = 0; c < D; ++c) Yj[c] = Ys(j, c);
        }
        F::vjp(t + TB::C(j) * h, Yj, in.th, in.par, kb[j], ybj, thb[r]);
#pragma unroll
        for (int c = 0; c < D; ++c) yb[c] += ybj[c];
        sfor<j>([&](auto L) {
          constexpr int l = decltype(L)::value;
          constexpr double a = TB::A(j, l);
          if constexpr (a != 0.0) {
#pragma unroll
            for (int c = 0; c < D; ++c) kb[l][c] = fma(h * a, ybj[c], kb[l][c]);
          }
        });
      }
    });
#pragma unroll
    for (int c = 0; c < D; ++c) lam[r][c] = yb[c];
  }
}

// Discrete adjoint, persistent like the forward solve.  A lane holds one
// trajectory and walks its tape backwards one segment at a time: in
// checkpoint mode a segment is the ckpt_every accepted steps after a
// checkpoint, replayed from it with the forward's own attempt function (so
// the same steps, bit for bit) while (t_n, h_n, y_n) of every accepted step
// goes to per-wave scratch; in store mode a segment is one step read from
// the tape.  The segment's steps are then reversed last to first, output
// node cotangents entering where their nodes fall.  Every lane of a wave
// works on a segment at the same time, so the replay and reverse phases
// never diverge; a lane whose trajectory is done takes the next one from the
// queue at the segment boundary.
//
// Between segments a lane keeps only a few integers in registers.  The
// running cotangents (lambda of y, and of theta) are in registers while a
// segment is reversed and in a per-wave buffer between segments, and the
// trajectory's inputs are reloaded for every segment; nothing floating-point
// is carried in registers across the divergent refill and finish code.
// Per-wave buffers are laid out [field][lane] (component stride 64), so a
// wave moves whole 512-byte rows; the stage points of the step being
// reversed live in LDS.
// STORE: the tape is in store mode (chosen by the host from ckpt_every), so
// the kernel holds no replay state at all.
constexpr int kStoreSegment = 32;

// A store-mode tape record (L consecutive doubles) held in registers as
// 16-byte vectors, so that a fetch lands in the variable itself and nothing
// copies it (a copy right after the fetch would wait for it); a record of
// odd length keeps its last value alone, so nothing past the record is read.
// The vectors claim only the 8-byte alignment a record has.
template <int L>
struct RecBuf {
  typedef double d2 __attribute__((ext_vector_type(2), aligned(8)));
  d2 v[L / 2];
  double tail;
  __device__ __forceinline__ void load(const double* p) {
#pragma unroll
    for (int k = 0; k < L / 2; ++k) v[k] = *reinterpret_cast<const d2*>(p + 2 * k);
    if constexpr (L % 2 != 0) tail = p[L - 1];
  }
  __device__ __forceinline__ double get(int i) const {
    if constexpr (L % 2 != 0) {
      if (i == L - 1) return tail;
    }
    return v[i / 2][i % 2];
  }
};
// Reverse of one step on a 16-lane group (one loss, no output seeds): the
// single-lane reverse_step component by component.  Lane c holds component
// c of the state, of the running cotangent and of every stage point and
// stage cotangent; the right-hand side is evaluated per component (row_f)
// and its vector-Jacobian product on the gathered stage point and stage
// cotangent in every lane, which keeps its component of the result and
// accumulates the same parameter cotangent as every other lane.  Sums run
// in the single lane's order, so the cotangents are bitwise its own.
template <class TB, class F>
__device__ __forceinline__ void group_reverse_step(const GroupCoef<TB>& cf, const Inputs<F>& in,
                                                   double t, double h, double yc, double& lam,
                                                   double (&thb)[F::P], int c) {
  constexpr int S = TB::S, D = F::D;
  double Ys[S], k[S];
#pragma unroll
  for (int j = 0; j < S; ++j) Ys[j] = k[j] = 0.0;
  Ys[0] = yc;
  k[0] = row_f<F>(t, yc, in.par, c);
  sfor<S - 1>([&](auto J1) {
    constexpr int j = decltype(J1)::value + 1;
    if constexpr (stage_feeds_step<TB>(j)) {
      double acc = 0.0;
      sfor<j>([&](auto L) {
        constexpr int l = decltype(L)::value;
        if constexpr (TB::A(j, l) != 0.0) acc = fma(cf.a[j][l], k[l], acc);
      });
      Ys[j] = fma(h, acc, yc);
      if constexpr (j < S - 1) k[j] = row_f<F>(t + cf.template node<j>() * h, Ys[j], in.par, c);
    }
  });
  double kb[S];
  sfor<S>([&](auto J) {
    constexpr int j = decltype(J)::value;
    kb[j] = (h * TB::B(j)) * lam;
  });
  double yb = lam;
  rfor<S>([&](auto J) {
    constexpr int j = decltype(J)::value;
    if constexpr (stage_feeds_step<TB>(j)) {
      double Yf[D], kbf[D], ybf[D];
      row_gather<D>(Ys[j], Yf);
      row_gather<D>(kb[j], kbf);
      F::vjp(t + TB::C(j) * h, Yf, in.th, in.par, kbf, ybf, thb);
      const double ybj = c < D ? pick<D>(ybf, c) : 0.0;
      yb += ybj;
      sfor<j>([&](auto L) {
        constexpr int l = decltype(L)::value;
        constexpr double a = TB::A(j, l);
        if constexpr (a != 0.0) kb[l] = fma(h * a, ybj, kb[l]);
      });
    }
  });
  lam = yb;
}

// The adjoint of the head of the queue order on 16-lane groups: one loss,
// final-state cotangents, store-mode tape.  Groups take queue positions
// [0, n_wide) from their own queue head (counters[3]), each walking its
// trajectory's tape from the last accepted step to the first (record n
// holds t_n and y_n, record n + 1 the length of step n) with the running
// cotangents in registers; the single lanes take the rest.  Results are
// written as one lane writes them: lane c component c of y0bar, lane 0 the
// parameter cotangents.
template <class TB, class F>
__device__ void vjp_group(const Params& P, const VjpParams& V) {
  constexpr int D = F::D, NP = F::P;
  const int lane = threadIdx.x & 63;
  const int c = lane & (kGroup - 1);
  const int first = lane & ~(kGroup - 1);  // the group's lane 0
  GroupCoef<TB> cf;
  cf.load();
  Inputs<F> in;
  int64_t idx = -1, ts = 0;
  bool live = false, ok = false, queue_empty = false;
  int32_t n = -1;  // the step to reverse next
  double lam = 0.0, thb[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) thb[q] = 0.0;
  auto finish = [&]() {
    if (c < D) V.y0bar[((int64_t)V.r0 * D + c) * P.n + idx] = ok ? lam : __builtin_nan("");
    if (c == 0) {
#pragma unroll
      for (int q = 0; q < NP; ++q)
        V.thetabar[((int64_t)V.r0 * NP + q) * P.n + idx] = ok ? thb[q] : __builtin_nan("");
    }
    live = false;
  };
  auto start = [&](int64_t i) {
    idx = i;
    live = true;
    ok = P.status[i] == ST_OK;
    ts = ok ? (int64_t)P.slot[i] : 0;
    lam = (V.ybar_final && c < D && V.R > 0) ? V.ybar_final[((int64_t)V.r0 * D + c) * P.n + i]
                                             : 0.0;
#pragma unroll
    for (int q = 0; q < NP; ++q) thb[q] = 0.0;
    double y_unused[D];
    load_inputs<F>(P, i, in, y_unused);
    n = P.n_acc[i] - 1;
    if (!ok || n < 0) finish();
  };
  for (;;) {
    if (!queue_empty) {
      const uint64_t idle = __ballot(!live && c == 0);  // one bit per idle group
      const int nidle = __popcll(idle);
      if (nidle > 0) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(P.counters + 3, (unsigned long long)nidle);
        base = first_lane(base);
        if (base + (unsigned long long)nidle >= (unsigned long long)P.n_wide) queue_empty = true;
        if (!live) {
          const uint64_t below = first ? (~0ull >> (64 - first)) : 0ull;
          const unsigned long long pos = base + __popcll(idle & below);
          if (pos < (unsigned long long)P.n_wide) {
            const int64_t id = P.order ? P.order[pos] : (int64_t)pos;
            if (id >= 0 && id < P.n) start(id);
          }
        }
      }
    }
    if (__ballot(live) == 0) {
      if (queue_empty) break;
      continue;
    }
    if (live) {
      const double* rec = P.tape + ((int64_t)ts * P.ckpt_cap + n) * store_record_len<F>();
      const double tn = rec[0];
      const double hn = rec[store_record_len<F>() + 1];
      const double yc = c < D ? rec[2 + c] : 0.0;
      group_reverse_step<TB, F>(cf, in, tn, hn, yc, lam, thb, c);
      --n;
      if (n < 0) finish();
    }
  }
}

template <class TB, class F, int R, bool NODES, bool STORE, bool WIDE = false>
__global__ void __launch_bounds__(256) vjp_kernel(Params P, VjpParams V) {
  if constexpr (WIDE) {
    static_assert(STORE && !NODES && R == 1 && F::D <= kGroup,
                  "groups reverse store-mode tapes of final-state losses");
    if ((int)blockIdx.x < P.wide_blocks) {  // uniform per workgroup
      vjp_group<TB, F>(P, V);
      return;
    }
  }
  constexpr int D = F::D, NP = F::P;
  constexpr int SREC = 2 + D;
  constexpr int AREC = D + NP;  // running cotangents of one loss
  const int lane = threadIdx.x & 63;
  // The per-wave scratch below is indexed from the first single-lane
  // workgroup: the group workgroups use none, and the host sizes the grid's
  // single-lane part, not the whole grid, to the scratch it has.
  const int64_t wave =
      (((int64_t)blockIdx.x - (WIDE ? P.wide_blocks : 0)) * blockDim.x + threadIdx.x) >> 6;
  constexpr bool store = STORE;
  // Steps per segment: the checkpoint interval, or in store mode a fixed
  // stretch of the tape (inputs, refill and bookkeeping once per segment).
  const int kseg = store ? kStoreSegment : P.ckpt_every;
  double* scr = V.scratch + (store ? 0 : wave * (int64_t)kseg * SREC * 64 + lane);
  // Stage points in dynamic LDS: (s - 1) d doubles per lane of the block.
  extern __shared__ double gs_lds[];
  double* ysc = gs_lds + threadIdx.x;
  const int ys = blockDim.x;
  double* ast = V.adj + wave * (int64_t)R * AREC * 64 + lane;
  auto LAM = [&](int r, int c) -> double& { return ast[(r * AREC + c) * 64]; };
  auto THB = [&](int r, int c) -> double& { return ast[(r * AREC + D + c) * 64]; };

  int64_t idx = -1, ts = 0;  // trajectory and its tape slot
  bool live = false, ok = false;
  bool queue_empty = false;  // wave-uniform
  int32_t N = 0, cseg = -1, kp = -1;

  auto gbar = [&](int r, int c, int kk) -> double {
    return (V.ybar_out && r < V.R)
               ? V.ybar_out[(((int64_t)(V.r0 + r) * D + c) * P.K + kk) * P.n + idx]
               : 0.0;
  };
  // Nodes at t0 read y0 directly; then the results leave the lane.
  auto finish = [&]() {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r < V.R) {
#pragma unroll
        for (int c = 0; c < D; ++c) {
          double l = LAM(r, c);
          for (int kk = kp; NODES && kk >= 0; --kk) l += gbar(r, c, kk);
          V.y0bar[((int64_t)(V.r0 + r) * D + c) * P.n + idx] = ok ? l : __builtin_nan("");
        }
#pragma unroll
        for (int c = 0; c < NP; ++c)
          V.thetabar[((int64_t)(V.r0 + r) * NP + c) * P.n + idx] =
              ok ? THB(r, c) : __builtin_nan("");
      }
    }
    live = false;
  };
  auto start = [&](int64_t i) {
    idx = i;
    live = true;
    N = P.n_acc[i];
    ok = P.status[i] == ST_OK;
    ts = ok ? (int64_t)P.slot[i] : 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int c = 0; c < D; ++c)
        LAM(r, c) = (V.ybar_final && r < V.R)
                        ? V.ybar_final[((int64_t)(V.r0 + r) * D + c) * P.n + i]
                        : 0.0;
#pragma unroll
      for (int c = 0; c < NP; ++c) THB(r, c) = 0.0;
    }
    kp = P.K - 1;
    cseg = (N + kseg - 1) / kseg - 1;
    if (!ok || cseg < 0) finish();
  };

  for (;;) {
    if (!queue_empty) {
      const uint64_t idle = __ballot(!live);
      const int nidle = __popcll(idle);
      if (nidle > 0) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(P.counters + 1, (unsigned long long)nidle);
        base = first_lane(base);
        if (base + (unsigned long long)nidle >= (unsigned long long)P.n) queue_empty = true;
        if (!live) {
          const unsigned long long pos = base + __popcll(idle & lanemask_lt());
          if (pos < (unsigned long long)P.n) {
            const int64_t id = P.order ? P.order[pos] : (int64_t)pos;
            if (id >= 0 && id < P.n) start(id);  // a bad permutation entry is skipped
          }
        }
      }
    }
    if (__ballot(live) == 0) {
      if (queue_empty) break;
      continue;
    }
    // This segment's inputs, on every lane (idle lanes read trajectory 0's,
    // in bounds and unused), so they are defined on every path.
    Traj<TB, F> s;
    {
      double y_unused[D];
      load_inputs<F>(P, live ? idx : 0, s.in, y_unused);
    }
    // Steps of this lane's current segment.
    const int m = live ? min(kseg, N - cseg * kseg) : 0;
    if constexpr (!store) {
      // Replay the segment from its checkpoint (idle lanes: record 0 of
      // trajectory 0, likewise unused).
      read_checkpoint<TB, F>(P, live ? ts : 0, live ? cseg : 0, s);
      s.nacc = cseg * kseg;
      s.nrej = 0;
      int j = 0;
      bool lost = false;  // the replay ended before m steps: not faithful
      while (__ballot(live && j < m && !lost) != 0) {
        // The forward's step limit bounds a replay that is not faithful.
        lost = lost | (live && j < m && (int64_t)s.nacc + s.nrej >= P.max_steps);
        if (live && j < m && !lost) {
          double* rec = scr + (int64_t)j * SREC * 64;
          rec[0] = s.t;
#pragma unroll
          for (int c = 0; c < D; ++c) rec[(2 + c) * 64] = s.y[c];
          const Attempt a = attempt<TB, F>(
              P, s, [&](const Traj<TB, F>&, double, double, const double (&)[D]) {});
          if (a.accepted) {
            rec[64] = a.h_used;
            ++j;
          }
          lost = a.finished && j < m;
        }
      }
      if (live) {
        // Bit-exact check against the next checkpoint, or for the last
        // segment against the forward's final state.
        bool same = !lost;
        if (!lost && (cseg + 1) * kseg < N) {
          const double* nxt = tape_record<TB, F>(P, ts, cseg + 1);
#pragma unroll
          for (int c = 0; c < D; ++c) same = same & (nxt[3 + c] == s.y[c]);
        } else if (!lost) {
#pragma unroll
          for (int c = 0; c < D; ++c) same = same & (P.y_final[(int64_t)c * P.n + idx] == s.y[c]);
        }
        if (!same) atomicAdd(P.counters + 2, 1ull);
        ok = ok & !lost;
      }
    }
    // Reverse the segment's steps, last to first.  The record of step n
    // holds (t_n, y_n) and, in store mode, h_{n-1} (replayed records hold
    // h_n), so each step reads one record; the next step's record is
    // fetched before this step's arithmetic.
    const int fs = store ? 1 : 64;  // field stride of a record
    auto record = [&](int jj) -> const double* {
      return store ? tape_record<TB, F>(P, ts, cseg * kseg + jj) : scr + (int64_t)jj * SREC * 64;
    };
    double nx_t = 0.0, nx_h = 0.0, nx_y[D];
    double h_carry = 0.0;  // store mode: h of the step about to be reversed
#pragma unroll
    for (int c = 0; c < D; ++c) nx_y[c] = 0.0;
    // The lane's first step of the segment (jj = m - 1) is read here, ahead
    // of the loop, so that the loop body has one path: each step takes the
    // record fetched one step earlier and issues the fetch of the next one,
    // which then stays in flight during the step's arithmetic (a first-step
    // branch inside the loop made the compiler wait for every outstanding
    // load, the new fetch included, at the top of each step).
    RecBuf<SREC> nxr;  // store mode: the record of the next step to reverse
    if (live && ok && m > 0) {
      const double* rec = record(m - 1);
      if constexpr (store) {
        nxr.load(rec);
        h_carry = tape_record<TB, F>(P, ts, cseg * kseg + m)[1];
      } else {
        nx_t = rec[0];
        nx_h = rec[fs];
#pragma unroll
        for (int c = 0; c < D; ++c) nx_y[c] = rec[(2 + c) * fs];
      }
    }
    // This segment's running cotangents (every lane reads its own slot, so
    // they are defined on every path).
    double lam[R][D], thb[R][NP];
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int c = 0; c < D; ++c) lam[r][c] = LAM(r, c);
#pragma unroll
      for (int c = 0; c < NP; ++c) thb[r][c] = THB(r, c);
    }
    // Take these loads to completion here: left outstanding into the loop,
    // the waits for them stay in the loop body and, memory counters being
    // in order, make every later step wait for its own prefetch as well.
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int c = 0; c < D; ++c) asm volatile("" : : "v"(lam[r][c]));
#pragma unroll
      for (int c = 0; c < NP; ++c) asm volatile("" : : "v"(thb[r][c]));
    }
    for (int jj = kseg - 1; jj >= 0; --jj) {
      const bool act = live && ok && jj < m;
      if (__ballot(act) == 0) continue;
      if (!act) continue;
      double tn, hn, yn[D];
      if constexpr (store) {
        tn = nxr.get(0);
        hn = h_carry;
#pragma unroll
        for (int c = 0; c < D; ++c) yn[c] = nxr.get(2 + c);
        h_carry = nxr.get(1);
        if (jj > 0) nxr.load(record(jj - 1));
      } else {
        tn = nx_t;
        hn = nx_h;
#pragma unroll
        for (int c = 0; c < D; ++c) yn[c] = nx_y[c];
        if (jj > 0) {
          const double* rec = record(jj - 1);
          nx_t = rec[0];
          nx_h = rec[fs];
#pragma unroll
          for (int c = 0; c < D; ++c) nx_y[c] = rec[(2 + c) * fs];
        }
      }
      const bool last_step = cseg * kseg + jj == N - 1;
      const double t_new = last_step ? s.in.t1 : tn + hn;
      auto no_seed = [](int, double(&)[TB::S][D], double(&)[D]) {};
      if constexpr (!NODES) {
        reverse_step<TB, F, R, NODES>(s.in, tn, hn, yn, lam, thb, false, no_seed, ysc, ys);
      } else {
        // The time of node kp is read for every step rather than carried
        // from the previous one: carried across the step's reverse pass, the
        // value (written inside the divergent node search below) was spilled
        // by the compiler in the join block ahead of the exec-mask restore,
        // so lanes that skipped the search kept a stale time and never
        // reversed their inner nodes.  The load hits the cache.
        double t_kp = node_time_or_ninf(P, kp, idx);
        // Nodes at the end of the step read y+ itself.
        while (kp >= 0 && t_kp == t_new) {
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) lam[r][c] += gbar(r, c, kp);
          --kp;
          t_kp = node_time_or_ninf(P, kp, idx);
        }
        // Nodes inside the step: indices kp, kp - 1, ..., k_lo + 1.
        int k_lo = kp;
        double t_lo = t_kp;
        while (k_lo >= 0 && t_lo > tn) {
          --k_lo;
          t_lo = k_lo >= 0 ? node_time(P, k_lo, idx) : -__builtin_inf();
        }
        if constexpr (TB::POLY_DENSE) {
          // All of them enter one reverse pass: their cotangents are linear
          // seeds of the stages, added while the stage cotangents are set
          // up (a short per-lane loop), so the step itself is reversed once.
          const int kp_top = kp;
          const bool any = kp > k_lo;
          auto seed = [&](int r, double (&kb)[TB::S][D], double (&yb)[D]) {
            for (int kq = kp_top; kq > k_lo; --kq) {
              const double sg = (node_time(P, kq, idx) - tn) / hn;
              double g[D];
#pragma unroll
              for (int c = 0; c < D; ++c) g[c] = gbar(r, c, kq);
              sfor<TB::S>([&](auto J) {
                constexpr int j = decltype(J)::value;
                double w = 0.0;
                rfor<TB::DEG>([&](auto Q) {
                  constexpr int qq = decltype(Q)::value;
                  w = fma(w, sg, TB::Bs(j, qq));
                });
                w *= sg * hn;
#pragma unroll
                for (int c = 0; c < D; ++c) kb[j][c] = fma(w, g[c], kb[j][c]);
              });
#pragma unroll
              for (int c = 0; c < D; ++c) yb[c] += g[c];
            }
          };
          reverse_step<TB, F, R, NODES>(s.in, tn, hn, yn, lam, thb, any, seed, ysc, ys);
          kp = k_lo;
        } else {
          // Shortened-step outputs: each is a full step of length sigma h
          // from y_n with its own stage points, so each takes a reverse pass
          // of its own, before the step itself; their cotangents of y_n are
          // summed with the step's.  One reverse_step call site: a lane
          // passes through its nodes, then its step.
          double acc[R][D];
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) acc[r][c] = 0.0;
          bool has;
          do {
            has = kp > k_lo;
            const double hq = has ? ((node_time(P, kp, idx) - tn) / hn) * hn : hn;
            double lz[R][D];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
              for (int c = 0; c < D; ++c) lz[r][c] = has ? gbar(r, c, kp) : lam[r][c];
            reverse_step<TB, F, R, NODES>(s.in, tn, hq, yn, lz, thb, false, no_seed, ysc, ys);
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
              for (int c = 0; c < D; ++c) {
                acc[r][c] += has ? lz[r][c] : 0.0;
                lam[r][c] = has ? lam[r][c] : lz[r][c] + acc[r][c];
              }
            kp -= has ? 1 : 0;
          } while (has);
        }
      }
    }
    // Segment done.
    if (live) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int c = 0; c < D; ++c) LAM(r, c) = lam[r][c];
#pragma unroll
        for (int c = 0; c < NP; ++c) THB(r, c) = thb[r][c];
      }
      cseg -= 1;
      if (!ok || cseg < 0) finish();
    }
  }
}

// ---------------------------------------------------------------------------
// Dense query: y(t_q) for Q times per trajectory: in store mode from the
// recorded step that contains t_q, otherwise by replaying from the last
// checkpoint before t_q (or from t0 without a tape).
template <class TB, class F>
__global__ void __launch_bounds__(256) dense_kernel(Params P, int32_t Q, const double* tq_all,
                                                    double* yq_all) {
  constexpr int D = F::D;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.n) return;
  Traj<TB, F> s;
  double y0[D];
  load_inputs<F>(P, i, s.in, y0);
  const int32_t st = P.status[i];
  const int32_t N = P.n_acc[i];
  const bool tape = P.ckpt_every > 0;
  const int64_t ts = (tape && st == ST_OK) ? (int64_t)P.slot[i] : 0;  // tape slot
  const int nseg = tape ? min((N + P.ckpt_every - 1) / P.ckpt_every, P.ckpt_cap) : 0;
  for (int q = 0; q < Q; ++q) {
    const double tq = tq_all[(int64_t)q * P.n + i];
    double out[D];
    bool done = false;
    if (st != ST_OK || !(tq >= s.in.t0) || !(tq <= s.in.t1)) {
#pragma unroll
      for (int c = 0; c < D; ++c) out[c] = __builtin_nan("");
      done = true;
    } else if (tq == s.in.t0) {
#pragma unroll
      for (int c = 0; c < D; ++c) out[c] = y0[c];
      done = true;
    }
    if (!done && P.store) {
      // Store mode: the step containing tq is on the tape; take it once.
      int lo = 0, hi = min(N, P.ckpt_cap - 1);
      while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (tape_record<TB, F>(P, ts, mid)[0] < tq)
          lo = mid;
        else
          hi = mid - 1;
      }
      const double* rec = tape_record<TB, F>(P, ts, lo);
      const double* nxt = tape_record<TB, F>(P, ts, lo + 1);
      if (lo >= N || lo + 1 >= P.ckpt_cap) {
#pragma unroll
        for (int c = 0; c < D; ++c) out[c] = __builtin_nan("");
      } else if (nxt[0] == tq) {
#pragma unroll
        for (int c = 0; c < D; ++c) out[c] = nxt[2 + c];
      } else {
        const double tn = rec[0], hn = nxt[1];
#pragma unroll
        for (int c = 0; c < D; ++c) s.y[c] = rec[2 + c];
        F::f(tn, s.y, s.in.par, s.k[0]);
        double yend[D];
        if constexpr (TB::POLY_DENSE) {
          rk_stages<TB, F>(s.in.par, tn, hn, s.y, s.k, yend);
        } else {
#pragma unroll
          for (int c = 0; c < D; ++c) yend[c] = nxt[2 + c];
        }
        dense_value<TB, F>(s.in.par, tn, hn, (tq - tn) / hn, yend, s.y, s.k, out);
      }
      done = true;
    }
    if (!done) {
      if (tape && nseg > 0) {
        // Last checkpoint strictly before tq.
        int lo = 0, hi = nseg - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) / 2;
          if (tape_record<TB, F>(P, ts, mid)[0] < tq)
            lo = mid;
          else
            hi = mid - 1;
        }
        read_checkpoint<TB, F>(P, ts, lo, s);
      } else {
#pragma unroll
        for (int c = 0; c < D; ++c) s.y[c] = y0[c];
        s.t = s.in.t0;
        s.err_prev2 = 1.0;
        s.nanrun = 0;
        F::f(s.t, s.y, s.in.par, s.k[0]);
        s.h = P.h0 > 0.0 ? dmin(P.h0, s.in.t1 - s.in.t0) : initial_step<TB, F>(s.in, s.y, s.k[0]);
      }
      s.nacc = 0;
      s.nrej = 0;
      for (int guard = 0; guard < 100000000 && !done; ++guard) {
        const Attempt a = attempt<TB, F>(
            P, s, [&](Traj<TB, F>& sb, double t_old, double hh, const double (&ys)[D]) {
              if (tq <= sb.t) {
                if (tq == sb.t) {
#pragma unroll
                  for (int c = 0; c < D; ++c) out[c] = sb.y[c];
                } else {
                  dense_value<TB, F>(sb.in.par, t_old, hh, (tq - t_old) / hh, sb.y, ys, sb.k, out);
                }
                done = true;
              }
            });
        if (a.finished && !done) {
#pragma unroll
          for (int c = 0; c < D; ++c) out[c] = __builtin_nan("");
          done = true;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < D; ++c) yq_all[((int64_t)c * Q + q) * P.n + i] = out[c];
  }
}

// ---------------------------------------------------------------------------
// Pointwise right-hand side and its VJP (for testing the hand-written
// transposes against forward-mode derivatives).
template <class F>
__global__ void __launch_bounds__(256) rhs_kernel(int64_t m, const double* t, const double* y,
                                                  const double* theta, double* f,
                                                  const double* kbar, double* ybar,
                                                  double* thetabar) {
  constexpr int D = F::D, NP = F::P;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double yy[D], th[NP], ff[D];
#pragma unroll
  for (int c = 0; c < D; ++c) yy[c] = y[(int64_t)c * m + i];
#pragma unroll
  for (int c = 0; c < NP; ++c) th[c] = theta[(int64_t)c * m + i];
  const typename F::Par par = F::prep(th);
  F::f(t[i], yy, par, ff);
  if (f) {
#pragma unroll
    for (int c = 0; c < D; ++c) f[(int64_t)c * m + i] = ff[c];
  }
  if (kbar && ybar && thetabar) {
    double kb[D], yb[D], tb[NP];
#pragma unroll
    for (int c = 0; c < D; ++c) kb[c] = kbar[(int64_t)c * m + i];
#pragma unroll
    for (int c = 0; c < NP; ++c) tb[c] = 0.0;
    F::vjp(t[i], yy, th, par, kb, yb, tb);
#pragma unroll
    for (int c = 0; c < D; ++c) ybar[(int64_t)c * m + i] = yb[c];
#pragma unroll
    for (int c = 0; c < NP; ++c) thetabar[(int64_t)c * m + i] = tb[c];
  }
}

}  // namespace gs
