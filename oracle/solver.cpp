// Oracle (test infrastructure only): the adaptive explicit Runge-Kutta
// integrator of the paper's Appendix "Numerical details", one trajectory at a
// time, in the order the paper states it:
//   stages Y_j, update y+ and error e                      (eq:rk)
//   scaled RMS error norm over the d components of y        (eq:errnorm)
//   accept iff ||e|| <= 1, next step from the controller    (eq:controller)
//   outputs inside an accepted step from the dense polynomial (eq:dense) or,
//   for Verner 7, from a shortened step from the start of the step
//   forward sensitivities: the same step applied to S with h fixed
//                                                          (eq:stage-sens)
// Readings where the paper is silent (safety factor, starting step, landing
// on t1, node tie-breaks, failure statuses) follow the design notes.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "dual.hpp"
#include "gso.hpp"
#include "rhs.hpp"

namespace gso {
namespace {

struct Ctrl {
  double safety, amin, amax, beta1, beta2;
  bool no_grow_after_reject;
};

// Scaled RMS norm of eq:errnorm with s_j = atol + rtol max(|y_j|, |y+_j|).
double err_norm(int d, const double* e, const double* y, const double* yn, double rtol,
                double atol) {
  double acc = 0.0;
  for (int j = 0; j < d; ++j) {
    double sj = atol + rtol * std::max(std::fabs(y[j]), std::fabs(yn[j]));
    double r = e[j] / sj;
    acc += r * r;
  }
  return std::sqrt(acc / d);
}

// Starting step of Hairer, Norsett & Wanner (1993, Sec. II.4): the paper does
// not give one.  Uses the RMS norm scaled by atol + rtol |y0|.
double initial_step(int rhs, int d, double t0, double t1, const double* y0, const double* f0,
                    const double* th, double rtol, double atol, int order) {
  double span = t1 - t0;
  double d0 = 0.0, d1 = 0.0;
  for (int j = 0; j < d; ++j) {
    double sc = atol + std::fabs(y0[j]) * rtol;
    d0 += (y0[j] / sc) * (y0[j] / sc);
    d1 += (f0[j] / sc) * (f0[j] / sc);
  }
  d0 = std::sqrt(d0 / d);
  d1 = std::sqrt(d1 / d);
  double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
  h0 = std::min(h0, span);
  double y1[MAXD], f1[MAXD];
  for (int j = 0; j < d; ++j) y1[j] = y0[j] + h0 * f0[j];
  rhs_eval<double>(rhs, t0 + h0, y1, th, f1);
  double d2 = 0.0;
  for (int j = 0; j < d; ++j) {
    double sc = atol + std::fabs(y0[j]) * rtol;
    double r = (f1[j] - f0[j]) / sc;
    d2 += r * r;
  }
  d2 = std::sqrt(d2 / d) / h0;
  double h1;
  if (d1 <= 1e-15 && d2 <= 1e-15)
    h1 = std::max(1e-6, h0 * 1e-3);
  else
    h1 = std::pow(0.01 / std::max(d1, d2), 1.0 / order);
  return std::min(std::min(100.0 * h0, h1), span);
}

// One explicit RK step of length h from (t, y) with k[0] = f(t, y) given:
// fills k[1..s-1], returns y+ (eq:rk).  The error weights are applied by the
// caller on the values only.
template <class T>
void rk_step(const Tableau& tb, int rhs, int d, double t, double h, const T* y, const T* th,
             T k[MAXS][MAXD], T* yplus) {
  for (int j = 1; j < tb.s; ++j) {
    T Y[MAXD];
    for (int i = 0; i < d; ++i) {
      T acc(0.0);
      for (int l = 0; l < j; ++l)
        if (tb.a[j][l] != 0.0) acc += tb.a[j][l] * k[l][i];
      Y[i] = y[i] + h * acc;
    }
    rhs_eval<T>(rhs, t + tb.c[j] * h, Y, th, k[j]);
  }
  for (int i = 0; i < d; ++i) {
    T acc(0.0);
    for (int j = 0; j < tb.s; ++j)
      if (tb.b[j] != 0.0) acc += tb.b[j] * k[j][i];
    yplus[i] = y[i] + h * acc;
  }
}

// Value at t + sigma h inside an accepted step (eq:dense), or the shortened
// step of length sigma h from the start of the step (Verner 7).
template <class T>
void dense_value(const Tableau& tb, int rhs, int d, double t, double h, double sigma,
                 const T* y, const T* th, T k[MAXS][MAXD], T* out) {
  if (tb.dense == DENSE_POLY) {
    double w[MAXS];
    for (int j = 0; j < tb.s; ++j) {
      double acc = 0.0, sp = sigma;
      for (int q = 0; q < tb.deg; ++q) {
        acc += tb.P[j][q] * sp;
        sp *= sigma;
      }
      w[j] = acc;
    }
    for (int i = 0; i < d; ++i) {
      T acc(0.0);
      for (int j = 0; j < tb.s; ++j)
        if (w[j] != 0.0) acc += w[j] * k[j][i];
      out[i] = y[i] + h * acc;
    }
  } else {
    T ks[MAXS][MAXD];
    for (int i = 0; i < d; ++i) ks[0][i] = k[0][i];
    rk_step<T>(tb, rhs, d, t, sigma * h, y, th, ks, out);
  }
}

struct Lane {
  const gso_problem* P;
  const Tableau* tb;
  int d, p, m;
  Ctrl ctrl;
};

// Gradient part of a value: 0 for doubles.
inline double gpart_of(double, int) { return 0.0; }
inline double gpart_of(const Dual& x, int s) { return gpart(x, s); }

template <class T>
void store_node(const Lane& L, int64_t i, int kk, const T* y) {
  const gso_problem& P = *L.P;
  int64_t n = P.n;
  for (int c = 0; c < L.d; ++c) {
    if (P.y_out) P.y_out[((int64_t)c * P.K + kk) * n + i] = val(y[c]);
    if (L.m > 0 && P.S_out)
      for (int s = 0; s < L.m; ++s)
        P.S_out[(((int64_t)c * L.m + s) * P.K + kk) * n + i] = gpart_of(y[c], s);
  }
}

template <class T>
void store_final(const Lane& L, int64_t i, const T* y) {
  const gso_problem& P = *L.P;
  int64_t n = P.n;
  for (int c = 0; c < L.d; ++c) {
    if (P.y_final) P.y_final[(int64_t)c * n + i] = val(y[c]);
    if (L.m > 0 && P.S_final)
      for (int s = 0; s < L.m; ++s) P.S_final[((int64_t)c * L.m + s) * n + i] = gpart_of(y[c], s);
  }
}

template <class T>
void set_inputs(const Lane& L, int64_t i, T* y, T* th);

template <>
void set_inputs<double>(const Lane& L, int64_t i, double* y, double* th) {
  const gso_problem& P = *L.P;
  for (int c = 0; c < L.d; ++c) y[c] = P.y0[(int64_t)c * P.n + i];
  for (int c = 0; c < L.p; ++c)
    th[c] = P.theta_stride ? P.theta[(int64_t)c * P.theta_stride + i] : P.theta[c];
}

// Seed the sensitivity columns: S(t0) = d y0 / d z, the identity on chosen
// initial-condition columns and zero on parameter columns (initial
// conditions are independent inputs).
template <>
void set_inputs<Dual>(const Lane& L, int64_t i, Dual* y, Dual* th) {
  double yv[MAXD], tv[MAXP];
  set_inputs<double>(L, i, yv, tv);
  for (int c = 0; c < L.d; ++c) y[c] = Dual(yv[c]);
  for (int c = 0; c < L.p; ++c) th[c] = Dual(tv[c]);
  for (int s = 0; s < L.m; ++s) {
    int col = L.P->cols[s];
    Dual* tgt = col < L.d ? &y[col] : &th[col - L.d];
    if (tgt->m == 0) {
      tgt->m = L.m;
      for (int q = 0; q < L.m; ++q) tgt->g[q] = 0.0;
    }
    tgt->g[s] = 1.0;
  }
}

template <class T>
void solve_one(const Lane& L, int64_t i) {
  const gso_problem& P = *L.P;
  const Tableau& tb = *L.tb;
  const int d = L.d;
  T y[MAXD], th[MAXP];
  set_inputs<T>(L, i, y, th);
  double thv[MAXP];
  for (int c = 0; c < L.p; ++c) thv[c] = val(th[c]);
  const double t0 = P.t0[P.t_stride ? i : 0];
  const double t1 = P.t1[P.t_stride ? i : 0];
  const double rtol = P.rtol[P.tol_stride ? i : 0];
  const double atol = P.atol[P.tol_stride ? i : 0];
  const double* tk = P.t_out;
  auto node_t = [&](int kk) {
    return P.t_out_stride ? tk[(int64_t)kk * P.t_out_stride + i] : tk[kk];
  };

  int32_t nacc = 0, nrej = 0, status = ST_OK;
  int kp = 0;  // next output node
  // Nodes at t0 take y0 (they belong to no step).
  while (kp < P.K && node_t(kp) <= t0) store_node<T>(L, i, kp++, y);

  const bool replay = P.h_replay != nullptr;
  const int32_t nrep = replay ? P.n_replay[i] : 0;

  bool y0fin = true;
  for (int c = 0; c < d; ++c) y0fin = y0fin && std::isfinite(val(y[c]));
  if (!y0fin) status = ST_NONFINITE;

  if (y0fin && t1 > t0 && !(replay && nrep == 0)) {
    T k[MAXS][MAXD];
    rhs_eval<T>(P.rhs, t0, y, th, k[0]);
    double t = t0;
    double h;
    if (replay) {
      h = P.h_replay[i * P.h_cap + 0];
    } else if (P.h0 > 0.0) {
      h = std::min(P.h0, t1 - t0);
    } else {
      double yv[MAXD], fv[MAXD];
      for (int c = 0; c < d; ++c) { yv[c] = val(y[c]); fv[c] = val(k[0][c]); }
      h = initial_step(P.rhs, d, t0, t1, yv, fv, thv, rtol, atol, tb.order);
    }
    const double b1 = L.ctrl.beta1 > 0.0 ? L.ctrl.beta1 : 1.0 / tb.order;
    double err_prev = 1.0;
    bool prev_rejected = false;
    int nan_streak = 0;
    for (;;) {
      if ((int64_t)nacc + nrej >= P.max_steps) { status = ST_MAX_STEPS; break; }
      bool last = false;
      if (replay) {
        h = P.h_replay[i * P.h_cap + nacc];
        last = (nacc == nrep - 1);
      } else if (t + h >= t1) {
        h = t1 - t;
        last = true;
      }
      T yn[MAXD];
      rk_step<T>(tb, P.rhs, d, t, h, y, th, k, yn);
      double e[MAXD], yv[MAXD], ynv[MAXD];
      for (int c = 0; c < d; ++c) {
        double acc = 0.0;
        for (int j = 0; j < tb.s; ++j)
          if (tb.bdiff[j] != 0.0) acc += tb.bdiff[j] * val(k[j][c]);
        e[c] = h * acc;
        yv[c] = val(y[c]);
        ynv[c] = val(yn[c]);
      }
      double en = err_norm(d, e, yv, ynv, rtol, atol);
      bool finite = std::isfinite(en);
      bool accept = replay ? true : (finite && en <= 1.0);
      double factor;
      if (!finite)
        factor = L.ctrl.amin;
      else if (en == 0.0)
        factor = L.ctrl.amax;
      else {
        double raw = L.ctrl.safety * std::pow(en, -b1);
        if (L.ctrl.beta2 != 0.0) raw *= std::pow(err_prev, L.ctrl.beta2);
        factor = std::min(L.ctrl.amax, std::max(L.ctrl.amin, raw));
      }
      if (accept) {
        const double t_new = last ? t1 : t + h;
        while (kp < P.K && node_t(kp) <= t_new) {
          double tq = node_t(kp);
          if (tq == t_new) {
            store_node<T>(L, i, kp, yn);
          } else {
            T out[MAXD];
            dense_value<T>(tb, P.rhs, d, t, h, (tq - t) / h, y, th, k, out);
            store_node<T>(L, i, kp, out);
          }
          ++kp;
        }
        if (P.h_rec && nacc < P.h_cap) P.h_rec[i * P.h_cap + nacc] = h;
        ++nacc;
        t = t_new;
        for (int c = 0; c < d; ++c) y[c] = yn[c];
        bool yfin = true;
        for (int c = 0; c < d; ++c) yfin = yfin && std::isfinite(val(y[c]));
        if (!yfin) { status = ST_NONFINITE; break; }
        err_prev = std::max(en, 1e-4);
        if (tb.fsal) {
          for (int c = 0; c < d; ++c) k[0][c] = k[tb.s - 1][c];
        } else {
          rhs_eval<T>(P.rhs, t, y, th, k[0]);
        }
        if (L.ctrl.no_grow_after_reject && prev_rejected) factor = std::min(1.0, factor);
        prev_rejected = false;
        nan_streak = 0;
        if (last) break;
      } else {
        ++nrej;
        prev_rejected = true;
        if (!finite) {
          if (++nan_streak >= 50) { status = ST_NONFINITE; break; }
        } else {
          nan_streak = 0;
        }
      }
      h = h * factor;
      if (!replay && std::fabs(h) < 16.0 * 2.220446049250313e-16 * std::max(std::fabs(t), 1.0)) {
        status = ST_DT_UNDERFLOW;
        break;
      }
    }
  }
  // Nodes a failed trajectory never reached are reported as NaN.
  for (; kp < P.K; ++kp) {
    T nanv[MAXD];
    for (int c = 0; c < d; ++c) nanv[c] = T(std::nan(""));
    store_node<T>(L, i, kp, nanv);
  }
  store_final<T>(L, i, y);
  if (P.n_acc) P.n_acc[i] = nacc;
  if (P.n_rej) P.n_rej[i] = nrej;
  if (P.status) P.status[i] = status;
}

}  // namespace
}  // namespace gso

extern "C" {

int gso_solve(const gso_problem* P) {
  using namespace gso;
  if (!P || P->n < 0 || P->rhs < 0 || P->rhs > 4 || P->tableau < 0 || P->tableau > 2) return 1;
  if (P->m < 0 || P->m > MAXM) return 1;
  Lane L;
  L.P = P;
  L.tb = &tableau(P->tableau);
  L.d = rhs_dim(P->rhs);
  L.p = rhs_nparam(P->rhs);
  L.m = P->m;
  L.ctrl = Ctrl{P->safety, P->alpha_min, P->alpha_max, P->beta1, P->beta2,
                P->no_grow_after_reject != 0};
  for (int s = 0; s < L.m; ++s)
    if (P->cols[s] < 0 || P->cols[s] >= L.d + L.p) return 1;
  int nt = P->nthreads > 0 ? P->nthreads : 1;
  if (nt > P->n) nt = (int)std::max<int64_t>(P->n, 1);
  auto work = [&](int w) {
    for (int64_t i = w; i < P->n; i += nt) {
      if (L.m > 0)
        solve_one<Dual>(L, i);
      else
        solve_one<double>(L, i);
    }
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

int gso_tableau(int id, int32_t* ints, double* dbl) {
  using namespace gso;
  if (id < 0 || id > 2) return 1;
  const Tableau& T = tableau(id);
  ints[0] = T.s; ints[1] = T.order; ints[2] = T.fsal ? 1 : 0; ints[3] = T.dense; ints[4] = T.deg;
  int s = T.s, o = 0;
  for (int j = 0; j < s; ++j) dbl[o++] = T.c[j];
  for (int j = 0; j < s; ++j)
    for (int l = 0; l < s; ++l) dbl[o++] = T.a[j][l];
  for (int j = 0; j < s; ++j) dbl[o++] = T.b[j];
  for (int j = 0; j < s; ++j) dbl[o++] = T.bdiff[j];
  for (int j = 0; j < s; ++j)
    for (int q = 0; q < 8; ++q) dbl[o++] = T.P[j][q];
  return 0;
}

int gso_rhs(int rhs, double t, const double* y, const double* theta, int32_t m,
            const int32_t* cols, double* f, double* J) {
  using namespace gso;
  if (rhs < 0 || rhs > 4 || m < 0 || m > MAXM) return 1;
  int d = rhs_dim(rhs), p = rhs_nparam(rhs);
  if (m == 0) {
    rhs_eval<double>(rhs, t, y, theta, f);
    return 0;
  }
  Dual yd[MAXD], thd[MAXP], fd[MAXD];
  for (int c = 0; c < d; ++c) yd[c] = Dual(y[c]);
  for (int c = 0; c < p; ++c) thd[c] = Dual(theta[c]);
  for (int s = 0; s < m; ++s) {
    if (cols[s] < 0 || cols[s] >= d + p) return 1;
    Dual* tgt = cols[s] < d ? &yd[cols[s]] : &thd[cols[s] - d];
    if (tgt->m == 0) { tgt->m = m; for (int q = 0; q < m; ++q) tgt->g[q] = 0.0; }
    tgt->g[s] = 1.0;
  }
  rhs_eval<Dual>(rhs, t, yd, thd, fd);
  for (int c = 0; c < d; ++c) {
    f[c] = fd[c].v;
    for (int s = 0; s < m; ++s) J[c * m + s] = gpart(fd[c], s);
  }
  return 0;
}

}  // extern "C"

namespace gso {
int rhs_dim(int id) {
  static const int d[5] = {2, 4, 6, 9, 3};
  return d[id];
}
int rhs_nparam(int id) {
  static const int p[5] = {1, 1, 3, 3, 4};
  return p[id];
}
}  // namespace gso
