// C ABI of the ensemble solver (declared in include/gradsolve.h): argument
// checks, workspace layout, dispatch to the kernel templates of
// gs_kernels.hpp for every (right-hand side, tableau) pair, and hipGraph
// capture.  No call allocates device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "gradsolve.h"
#include "gs_kernels.hpp"

namespace {

using gs::Params;
using gs::VjpParams;

constexpr int kNumRhs = 5;
constexpr int kNumTab = 3;
constexpr int64_t kAdjMaxLanes = 131072;  // adjoint lanes on one GPU (2 waves per SIMD)
constexpr size_t kCounterBytes = 256;
constexpr int kVjpMaxR = 2;               // losses per adjoint launch

int rhs_dim(int r) {
  static const int d[kNumRhs] = {gs::Harmonic::D, gs::Kepler::D, gs::LogHalo::D,
                                 gs::SpinPrec::D, gs::Quint::D};
  return d[r];
}
int rhs_np(int r) {
  static const int p[kNumRhs] = {gs::Harmonic::P, gs::Kepler::P, gs::LogHalo::P,
                                 gs::SpinPrec::P, gs::Quint::P};
  return p[r];
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t tape_off, tape_bytes, scratch_off, scratch_bytes, total;
  int64_t adj_lanes;
};

Layout layout_of(const gs_solve_args* a) {
  Layout L;
  const int d = rhs_dim(a->rhs);
  L.tape_off = kCounterBytes;
  L.tape_bytes = 0;
  L.scratch_bytes = 0;
  L.adj_lanes = 0;
  if (a->ckpt_every > 0) {
    L.tape_bytes = (size_t)a->n * (size_t)a->ckpt_capacity * (size_t)(3 + 2 * d) * 8;
    L.adj_lanes = std::min<int64_t>((a->n + 255) / 256 * 256, kAdjMaxLanes);
    L.scratch_bytes = (size_t)L.adj_lanes * (size_t)a->ckpt_every * (size_t)(2 + d) * 8;
  }
  L.scratch_off = align256(L.tape_off + L.tape_bytes);
  L.total = L.scratch_off + L.scratch_bytes;
  return L;
}

// Host-side argument checks (everything that needs no device memory).
gs_status check_args(const gs_solve_args* a) {
  if (!a) return GS_ERR_INVALID;
  if (a->rhs < 0 || a->rhs >= kNumRhs || a->tableau < 0 || a->tableau >= kNumTab)
    return GS_ERR_INVALID;
  if (a->n < 0 || a->d != rhs_dim(a->rhs) || a->p != rhs_np(a->rhs)) return GS_ERR_INVALID;
  if (a->n > (int64_t)1 << 31) return GS_ERR_UNSUPPORTED;
  if (a->n == 0) return GS_OK;
  if (!a->y0 || !a->theta || !a->t0 || !a->t1 || !a->rtol || !a->atol) return GS_ERR_INVALID;
  if (!a->y_final || !a->n_accepted || !a->n_rejected || !a->status) return GS_ERR_INVALID;
  if (a->theta_stride != 0 && a->theta_stride != a->n) return GS_ERR_INVALID;
  if (a->t_stride != 0 && a->t_stride != 1) return GS_ERR_INVALID;
  if (a->tol_stride != 0 && a->tol_stride != 1) return GS_ERR_INVALID;
  if (a->K < 0) return GS_ERR_INVALID;
  if (a->K > 0 && (!a->t_out || !a->y_out)) return GS_ERR_INVALID;
  if (a->K > 0 && a->t_out_stride != 0 && a->t_out_stride != a->n) return GS_ERR_INVALID;
  if (a->ckpt_every < 0 || a->ckpt_capacity < 0) return GS_ERR_INVALID;
  if (a->ckpt_every > 0 && a->ckpt_capacity < 1) return GS_ERR_INVALID;
  if (a->schedule != GS_SCHED_QUEUE && a->schedule != GS_SCHED_STATIC) return GS_ERR_INVALID;
  if (a->block != 0 && (a->block < 64 || a->block > 256 || a->block % 64 != 0))
    return GS_ERR_INVALID;
  if (a->grid < 0) return GS_ERR_INVALID;
  if (a->refill < 0 || a->refill > 64) return GS_ERR_INVALID;
  const gs_controller& c = a->ctrl;
  if (!(c.safety > 0.0) || !(c.alpha_min > 0.0) || !(c.alpha_max >= 1.0) ||
      !(c.alpha_min <= 1.0))
    return GS_ERR_INVALID;
  if (!a->workspace) return GS_ERR_WORKSPACE;
  if (a->workspace_bytes < layout_of(a).total) return GS_ERR_WORKSPACE;
  if (((uintptr_t)a->workspace & 255) != 0) return GS_ERR_WORKSPACE;
  return GS_OK;
}

Params make_params(const gs_solve_args* a) {
  Params P;
  std::memset(&P, 0, sizeof P);
  P.n = a->n;
  P.y0 = a->y0;
  P.theta = a->theta;
  P.theta_stride = a->theta_stride;
  P.t0 = a->t0;
  P.t1 = a->t1;
  P.t_stride = a->t_stride;
  P.rtol = a->rtol;
  P.atol = a->atol;
  P.tol_stride = a->tol_stride;
  P.K = a->K;
  P.t_out = a->t_out;
  P.t_out_stride = a->t_out_stride;
  P.y_out = a->y_out;
  P.y_final = a->y_final;
  P.n_acc = a->n_accepted;
  P.n_rej = a->n_rejected;
  P.status = a->status;
  P.max_steps = a->max_steps > 0 ? a->max_steps : 10000000;
  P.h0 = a->h0;
  P.safety = a->ctrl.safety;
  P.amin = a->ctrl.alpha_min;
  P.amax = a->ctrl.alpha_max;
  P.beta1 = a->ctrl.beta1;
  P.beta2 = a->ctrl.beta2;
  P.ckpt_every = a->ckpt_every;
  P.ckpt_cap = a->ckpt_capacity;
  const Layout L = layout_of(a);
  char* ws = static_cast<char*>(a->workspace);
  P.counters = reinterpret_cast<unsigned long long*>(ws);
  P.tape = a->ckpt_every > 0 ? reinterpret_cast<double*>(ws + L.tape_off) : nullptr;
  P.order = a->order;
  P.refill = a->refill > 0 ? a->refill : 16;
  P.sched_static = a->schedule == GS_SCHED_STATIC ? 1 : 0;
  P.fast_ctrl = (a->ctrl.beta1 <= 0.0 && a->ctrl.beta2 == 0.0 && a->ctrl.alpha_max <= 100.0 &&
                 a->ctrl.alpha_min >= 0.01)
                    ? 1
                    : 0;
  return P;
}

int num_cus() {
  static int cus = 0;
  static std::once_flag once;
  std::call_once(once, [] {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 0;
  });
  return cus > 0 ? cus : 256;
}

// Kernel launchers for one (tableau, right-hand side) pair.
struct Ops {
  const void* solve_fn;
  void (*solve)(const Params&, int grid, int block, hipStream_t);
  void (*vjp)(const Params&, const VjpParams&, int grid, int block, hipStream_t);
  void (*dense)(const Params&, int32_t Q, const double*, double*, int grid, int block,
                hipStream_t);
};

template <class TB, class F>
void launch_solve(const Params& P, int grid, int block, hipStream_t s) {
  if (P.K > 0) {
    if (P.ckpt_every > 0)
      hipLaunchKernelGGL((gs::solve_kernel<TB, F, true, true>), dim3(grid), dim3(block), 0, s, P);
    else
      hipLaunchKernelGGL((gs::solve_kernel<TB, F, true, false>), dim3(grid), dim3(block), 0, s, P);
  } else {
    if (P.ckpt_every > 0)
      hipLaunchKernelGGL((gs::solve_kernel<TB, F, false, true>), dim3(grid), dim3(block), 0, s, P);
    else
      hipLaunchKernelGGL((gs::solve_kernel<TB, F, false, false>), dim3(grid), dim3(block), 0, s,
                         P);
  }
}
template <class TB, class F>
void launch_vjp(const Params& P, const VjpParams& V, int grid, int block, hipStream_t s) {
  if (V.R >= 2)
    hipLaunchKernelGGL((gs::vjp_kernel<TB, F, 2>), dim3(grid), dim3(block), 0, s, P, V);
  else
    hipLaunchKernelGGL((gs::vjp_kernel<TB, F, 1>), dim3(grid), dim3(block), 0, s, P, V);
}
template <class TB, class F>
void launch_dense(const Params& P, int32_t Q, const double* tq, double* yq, int grid, int block,
                  hipStream_t s) {
  hipLaunchKernelGGL((gs::dense_kernel<TB, F>), dim3(grid), dim3(block), 0, s, P, Q, tq, yq);
}
template <class TB, class F>
Ops make_ops() {
  return Ops{reinterpret_cast<const void*>(&gs::solve_kernel<TB, F, true, true>),
             &launch_solve<TB, F>,
             &launch_vjp<TB, F>, &launch_dense<TB, F>};
}
template <class F>
void ops_row(Ops* row) {
  row[GS_DOPRI5] = make_ops<gs::Dopri5, F>();
  row[GS_TSIT5] = make_ops<gs::Tsit5, F>();
  row[GS_VERNER7] = make_ops<gs::Verner7, F>();
}
const Ops& ops(int rhs, int tab) {
  static Ops table[kNumRhs][kNumTab];
  static std::once_flag once;
  std::call_once(once, [] {
    ops_row<gs::Harmonic>(table[GS_RHS_HARMONIC]);
    ops_row<gs::Kepler>(table[GS_RHS_KEPLER]);
    ops_row<gs::LogHalo>(table[GS_RHS_LOGHALO]);
    ops_row<gs::SpinPrec>(table[GS_RHS_SPINPREC]);
    ops_row<gs::Quint>(table[GS_RHS_QUINT]);
  });
  return table[rhs][tab];
}

// Grid of the forward launch: static mode covers n lanes; the persistent
// queue mode fills every CU to its occupancy limit but never launches more
// lanes than trajectories.
void solve_shape(const gs_solve_args* a, int* grid, int* block) {
  const int b = a->block > 0 ? a->block : 256;
  const int64_t need = (a->n + b - 1) / b;
  if (a->schedule == GS_SCHED_STATIC) {
    *grid = (int)need;
  } else if (a->grid > 0) {
    *grid = (int)std::min<int64_t>(a->grid, need);
  } else {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ops(a->rhs, a->tableau).solve_fn,
                                                     b, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    *grid = (int)std::min<int64_t>((int64_t)per_cu * num_cus(), need);
  }
  *block = b;
}

gs_status launch_solve_all(const gs_solve_args* a) {
  hipStream_t s = static_cast<hipStream_t>(a->stream);
  const Params P = make_params(a);
  hipLaunchKernelGGL(gs::reset_counters_kernel, dim3(1), dim3(64), 0, s, P.counters, 4);
  int grid = 0, block = 0;
  solve_shape(a, &grid, &block);
  ops(a->rhs, a->tableau).solve(P, grid, block, s);
  return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

}  // namespace

struct gs_graph {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

extern "C" {

void gs_default_args(gs_solve_args* a) {
  if (!a) return;
  std::memset(a, 0, sizeof *a);
  a->ctrl.safety = 0.9;
  a->ctrl.alpha_min = 0.2;
  a->ctrl.alpha_max = 5.0;
  a->ctrl.beta1 = 0.0;
  a->ctrl.beta2 = 0.0;
  a->max_steps = 10000000;
  a->schedule = GS_SCHED_QUEUE;
}

size_t gs_workspace_bytes(const gs_solve_args* a) {
  if (!a || a->rhs < 0 || a->rhs >= kNumRhs || a->n < 0 || a->ckpt_every < 0 ||
      a->ckpt_capacity < 0)
    return 0;
  return layout_of(a).total;
}

gs_status gs_solve(const gs_solve_args* a) {
  const gs_status st = check_args(a);
  if (st != GS_OK || a->n == 0) return st;
  return launch_solve_all(a);
}

gs_status gs_solve_vjp(const gs_solve_args* fwd, const gs_vjp_args* v) {
  gs_status st = check_args(fwd);
  if (st != GS_OK) return st;
  if (!v || v->R < 1 || v->R > 8 || !v->y0bar || !v->thetabar) return GS_ERR_INVALID;
  if (v->ybar_out && fwd->K == 0) return GS_ERR_INVALID;
  if (fwd->ckpt_every <= 0) return GS_ERR_NO_TAPE;
  if (v->block != 0 && (v->block < 64 || v->block > 256 || v->block % 64 != 0))
    return GS_ERR_INVALID;
  if (fwd->n == 0) return GS_OK;
  const Layout L = layout_of(fwd);
  const int block = v->block > 0 ? v->block : 256;
  int grid = (int)(L.adj_lanes / block);
  if (v->grid > 0) grid = std::min(grid, v->grid);
  if (grid < 1) return GS_ERR_INVALID;
  hipStream_t s = static_cast<hipStream_t>(v->stream);
  const Params P = make_params(fwd);
  VjpParams V;
  V.R_total = v->R;
  V.ybar_out = v->ybar_out;
  V.ybar_final = v->ybar_final;
  V.y0bar = v->y0bar;
  V.thetabar = v->thetabar;
  V.scratch = reinterpret_cast<double*>(static_cast<char*>(fwd->workspace) + L.scratch_off);
  hipLaunchKernelGGL(gs::reset_counters_kernel, dim3(1), dim3(64), 0, s, P.counters + 2, 1);
  for (int r0 = 0; r0 < v->R; r0 += kVjpMaxR) {
    V.r0 = r0;
    V.R = std::min(kVjpMaxR, v->R - r0);
    hipLaunchKernelGGL(gs::reset_counters_kernel, dim3(1), dim3(64), 0, s, P.counters + 1, 1);
    ops(fwd->rhs, fwd->tableau).vjp(P, V, grid, block, s);
  }
  return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

gs_status gs_dense_eval(const gs_solve_args* fwd, int32_t Q, const double* t_query,
                        double* y_query, void* stream) {
  const gs_status st = check_args(fwd);
  if (st != GS_OK) return st;
  if (Q < 0 || (Q > 0 && (!t_query || !y_query))) return GS_ERR_INVALID;
  if (Q == 0 || fwd->n == 0) return GS_OK;
  const int block = 256;
  const int grid = (int)((fwd->n + block - 1) / block);
  const Params P = make_params(fwd);
  ops(fwd->rhs, fwd->tableau)
      .dense(P, Q, t_query, y_query, grid, block, static_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

gs_status gs_rhs_eval(int32_t rhs, int64_t m, const double* t, const double* y,
                      const double* theta, double* f, const double* kbar, double* ybar,
                      double* thetabar, void* stream) {
  if (rhs < 0 || rhs >= kNumRhs || m < 0) return GS_ERR_INVALID;
  if (m == 0) return GS_OK;
  if (!t || !y || !theta) return GS_ERR_INVALID;
  const bool want_vjp = kbar || ybar || thetabar;
  if (want_vjp && !(kbar && ybar && thetabar)) return GS_ERR_INVALID;
  const int block = 256;
  const int grid = (int)((m + block - 1) / block);
  hipStream_t s = static_cast<hipStream_t>(stream);
  switch (rhs) {
    case GS_RHS_HARMONIC:
      hipLaunchKernelGGL(gs::rhs_kernel<gs::Harmonic>, dim3(grid), dim3(block), 0, s, m, t, y,
                         theta, f, kbar, ybar, thetabar);
      break;
    case GS_RHS_KEPLER:
      hipLaunchKernelGGL(gs::rhs_kernel<gs::Kepler>, dim3(grid), dim3(block), 0, s, m, t, y,
                         theta, f, kbar, ybar, thetabar);
      break;
    case GS_RHS_LOGHALO:
      hipLaunchKernelGGL(gs::rhs_kernel<gs::LogHalo>, dim3(grid), dim3(block), 0, s, m, t, y,
                         theta, f, kbar, ybar, thetabar);
      break;
    case GS_RHS_SPINPREC:
      hipLaunchKernelGGL(gs::rhs_kernel<gs::SpinPrec>, dim3(grid), dim3(block), 0, s, m, t, y,
                         theta, f, kbar, ybar, thetabar);
      break;
    default:
      hipLaunchKernelGGL(gs::rhs_kernel<gs::Quint>, dim3(grid), dim3(block), 0, s, m, t, y,
                         theta, f, kbar, ybar, thetabar);
      break;
  }
  return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

gs_status gs_graph_create(const gs_solve_args* a, gs_graph** out) {
  if (!out) return GS_ERR_INVALID;
  *out = nullptr;
  const gs_status st = check_args(a);
  if (st != GS_OK) return st;
  if (a->n == 0) return GS_ERR_INVALID;
  hipStream_t cap;
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return GS_ERR_HIP;
  gs_solve_args c = *a;
  c.stream = cap;
  gs_status rc = GS_OK;
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rc = GS_ERR_HIP;
  } else {
    rc = launch_solve_all(&c);
    if (hipStreamEndCapture(cap, &graph) != hipSuccess) rc = GS_ERR_HIP;
  }
  hipGraphExec_t exec = nullptr;
  if (rc == GS_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
    rc = GS_ERR_HIP;
  (void)hipStreamDestroy(cap);
  if (rc != GS_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  gs_graph* g = new gs_graph{graph, exec};
  *out = g;
  return GS_OK;
}

gs_status gs_graph_launch(gs_graph* g, void* stream) {
  if (!g) return GS_ERR_INVALID;
  return hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? GS_OK
                                                                                 : GS_ERR_HIP;
}

void gs_graph_destroy(gs_graph* g) {
  if (!g) return;
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  delete g;
}

const char* gs_status_string(gs_status s) {
  switch (s) {
    case GS_OK: return "ok";
    case GS_ERR_INVALID: return "invalid argument";
    case GS_ERR_UNSUPPORTED: return "unsupported request";
    case GS_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case GS_ERR_HIP: return "HIP runtime error";
    case GS_ERR_NO_TAPE: return "no gradient tape (ckpt_every == 0)";
  }
  return "unknown status";
}

const char* gs_version(void) { return "0.1.0"; }

}  // extern "C"
