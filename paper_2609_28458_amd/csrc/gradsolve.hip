// C ABI of the ensemble solver (declared in include/gradsolve.h): argument
// checks, workspace layout, dispatch to the kernel templates of
// gs_kernels.hpp for every (right-hand side, tableau) pair, and hipGraph
// capture.  No call allocates device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "gradsolve.h"
#include "gs_de.hpp"
#include "gs_kernels.hpp"
#include "gs_ops.hpp"
#include "gs_order.hpp"

namespace {

using gs::Params;
using gs::VjpParams;

constexpr int kNumRhs = 9;      // five explicit right-hand sides, then the four stiff ones
constexpr int kNumTab = 4;      // three explicit pairs, then Rodas4
constexpr int kNumExplicitRhs = 5;
constexpr int kNumExplicitTab = 3;
constexpr int64_t kAdjMaxLanes = 131072;  // adjoint lanes on one GPU (2 waves per SIMD)
constexpr size_t kCounterBytes = 256;
// Losses per adjoint launch.  Each further loss is another launch; one loss
// per lane keeps the adjoint kernels small enough to compile without
// kilobytes of register spills for the largest right-hand sides.
constexpr int kVjpMaxR = 1;
constexpr int kSensMaxCols = 16;          // sensitivity columns per call

// Clears the queue and replay counters at the head of the workspace (a
// kernel rather than a memset, so a captured graph holds no memset node).
__global__ void reset_counters_kernel(unsigned long long* c, int n) {
  if ((int)threadIdx.x < n) c[threadIdx.x] = 0ull;
}
// Adjoint queue heads: single lanes start after the head the groups reverse.
__global__ void reset_vjp_queues_kernel(unsigned long long* c, long long n_wide) {
  if (threadIdx.x == 0) c[1] = (unsigned long long)n_wide;
  if (threadIdx.x == 1) c[3] = 0ull;
}
// Forward queue heads: single lanes start after the wide head of the order.
__global__ void reset_queues_kernel(unsigned long long* c, long long n_wide) {
  if (threadIdx.x < 4) c[threadIdx.x] = threadIdx.x == 0 ? (unsigned long long)n_wide : 0ull;
}

// Marks every trajectory as not run before a solve with a caller-given queue
// order: an index the order misses keeps GS_TRAJ_NOT_RUN (the solve kernels
// overwrite the status of every trajectory they take).
__global__ void fill_status_kernel(int32_t* status, int64_t n, int32_t v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    status[i] = v;
}
// NaN into the cotangents of the losses of one adjoint call, before an
// adjoint with a caller-given order (so a missed index reads NaN).
__global__ void fill_nan_kernel(double* a, int64_t m) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride)
    a[i] = __builtin_nan("");
}
int fill_grid(int64_t m) { return (int)std::min<int64_t>((m + 255) / 256, 4096); }

int rhs_dim(int r) {
  static const int d[kNumExplicitRhs] = {gs::Harmonic::D, gs::Kepler::D, gs::LogHalo::D,
                                         gs::SpinPrec::D, gs::Quint::D};
  return r < kNumExplicitRhs ? d[r] : gs_host::stiff_dim(r);
}
int rhs_np(int r) {
  static const int p[kNumExplicitRhs] = {gs::Harmonic::P, gs::Kepler::P, gs::LogHalo::P,
                                         gs::SpinPrec::P, gs::Quint::P};
  return r < kNumExplicitRhs ? p[r] : gs_host::stiff_np(r);
}

// The stiff path: Rodas4 on a stiff right-hand side (check_args requires both
// or neither).
bool is_stiff(const gs_solve_args* a) { return a->tableau == GS_RODAS4; }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t tape_off, tape_bytes, scratch_off, scratch_bytes, adj_off, adj_bytes, pending_off,
      pending_bytes, slot_off, slot_bytes, total;
  int64_t adj_lanes;
};

// Outputs of the plain solve of an explicit pair (K > 0) are deferred to the
// output kernel: pending [K][n][2 + d] doubles.  `defer` false (the
// no-allocation entry point, when they do not fit) keeps a polynomial pair's
// outputs in the solve kernel; a pair without a polynomial always defers.
bool defers_outputs(const gs_solve_args* a, bool defer) {
  return a->K > 0 && a->rhs >= 0 && a->rhs < kNumExplicitRhs &&
         (defer || a->tableau == GS_VERNER7);
}

Layout layout_of(const gs_solve_args* a, bool defer = true) {
  Layout L;
  const int d = rhs_dim(a->rhs);
  L.tape_off = kCounterBytes;
  L.tape_bytes = 0;
  L.scratch_bytes = 0;
  L.adj_bytes = 0;
  L.adj_lanes = 0;
  if (a->ckpt_every > 0) {
    // Store mode (ckpt_every == 1) records (t, h, y) of every accepted step
    // and needs no replay scratch; checkpoint mode records the controller
    // state every ckpt_every steps and replays segments into scratch.
    const bool store = a->ckpt_every == 1;
    L.tape_bytes = (size_t)a->n * (size_t)a->ckpt_capacity * (size_t)(store ? 2 + d : 3 + 2 * d) * 8;
    L.adj_lanes = std::min<int64_t>((a->n + 255) / 256 * 256, kAdjMaxLanes);
    L.scratch_bytes = store ? 0 : (size_t)L.adj_lanes * (size_t)a->ckpt_every * (size_t)(2 + d) * 8;
    // Running cotangents of y and theta for the losses of one launch.
    L.adj_bytes = (size_t)L.adj_lanes * (size_t)kVjpMaxR * (size_t)(d + rhs_np(a->rhs)) * 8;
  }
  L.scratch_off = align256(L.tape_off + L.tape_bytes);
  L.adj_off = align256(L.scratch_off + L.scratch_bytes);
  L.pending_off = align256(L.adj_off + L.adj_bytes);
  L.pending_bytes =
      defers_outputs(a, defer) ? (size_t)(2 + d) * (size_t)a->K * (size_t)a->n * 8 : 0;
  // With a tape, each trajectory's tape slot (the queue position the
  // forward took it from), read by the adjoint and dense queries.
  L.slot_off = align256(L.pending_off + L.pending_bytes);
  L.slot_bytes = a->ckpt_every > 0 ? (size_t)a->n * 4 : 0;
  L.total = L.slot_off + L.slot_bytes;
  return L;
}

// Host-side argument checks (everything that needs no device memory).
gs_status check_args(const gs_solve_args* a, bool defer = true) {
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
  if (a->wide < 0) return GS_ERR_INVALID;
  if (a->out_layout != 0 && a->out_layout != 1) return GS_ERR_INVALID;
  if (a->wide > 0 && a->schedule != GS_SCHED_QUEUE)
    return GS_ERR_UNSUPPORTED;
  const gs_controller& c = a->ctrl;
  if (!(c.safety > 0.0) || !(c.alpha_min > 0.0) || !(c.alpha_max >= 1.0) ||
      !(c.alpha_min <= 1.0))
    return GS_ERR_INVALID;
  if ((a->rhs >= kNumExplicitRhs) != is_stiff(a)) return GS_ERR_UNSUPPORTED;
  if (is_stiff(a) && (a->ckpt_every > 0 || a->wide > 0 || a->out_layout != 0 || c.beta1 > 0.0 ||
                      c.beta2 != 0.0))
    return GS_ERR_UNSUPPORTED;
  if (!a->workspace) return GS_ERR_WORKSPACE;
  if (a->workspace_bytes < layout_of(a, defer).total) return GS_ERR_WORKSPACE;
  if (((uintptr_t)a->workspace & 255) != 0) return GS_ERR_WORKSPACE;
  return GS_OK;
}

// Order nu of the propagated solution (the controller exponent is 1/nu).
int tab_order(int tab) {
  static const int nu[kNumTab] = {5, 5, 7, 4};
  return (tab >= 0 && tab < kNumTab) ? nu[tab] : 7;
}

// The kernels' fast controller root clamps the squared norm to [1e-30,
// 1e30] (the norm to [1e-15, 1e15]) before taking safety * ||e||^(-1/nu).
// That changes no factor exactly when the clamped extremes already lie
// outside [alpha_min, alpha_max]: safety * 1e15^(1/nu) >= alpha_max and
// safety * 1e-15^(1/nu) <= alpha_min.  Otherwise, and for the PI form or
// another exponent, the kernels take pow.
bool fast_controller_exact(const gs_solve_args* a) {
  const gs_controller& c = a->ctrl;
  if (!(c.beta1 <= 0.0) || c.beta2 != 0.0) return false;
  const double g = std::pow(10.0, 15.0 / tab_order(a->tableau));
  return c.safety * g >= c.alpha_max && c.safety / g <= c.alpha_min;
}

Params make_params(const gs_solve_args* a, bool defer = true) {
  Params P;
  std::memset(&P, 0, sizeof P);
  P.n = a->n;
  P.out_layout = a->out_layout;
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
  P.store = a->ckpt_every == 1 ? 1 : 0;
  const Layout L = layout_of(a, defer);
  char* ws = static_cast<char*>(a->workspace);
  P.counters = reinterpret_cast<unsigned long long*>(ws);
  P.tape = a->ckpt_every > 0 ? reinterpret_cast<double*>(ws + L.tape_off) : nullptr;
  P.pending = L.pending_bytes ? reinterpret_cast<double*>(ws + L.pending_off) : nullptr;
  P.slot = L.slot_bytes ? reinterpret_cast<int32_t*>(ws + L.slot_off) : nullptr;
  P.order = a->order;
  P.refill = a->refill > 0 ? a->refill : 8;
  P.sched_static = a->schedule == GS_SCHED_STATIC ? 1 : 0;
  P.n_wide = std::min<int64_t>(a->wide, a->n);
  P.wide_blocks = 0;  // set with the launch shape
  P.fast_ctrl = fast_controller_exact(a) ? 1 : 0;
  return P;
}

size_t max_lds_per_block() {
  static int bytes = 0;
  static std::once_flag once;
  std::call_once(once, [] {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      bytes = 0;
  });
  return bytes > 0 ? (size_t)bytes : 65536;
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

using gs_host::Ops;

const Ops& ops(int rhs, int tab) {
  static Ops table[kNumRhs][kNumTab];
  static std::once_flag once;
  std::call_once(once, [] {
    gs_host::ops_row_harmonic(table[GS_RHS_HARMONIC]);
    gs_host::ops_row_kepler(table[GS_RHS_KEPLER]);
    gs_host::ops_row_loghalo(table[GS_RHS_LOGHALO]);
    gs_host::ops_row_spinprec(table[GS_RHS_SPINPREC]);
    gs_host::ops_row_quint(table[GS_RHS_QUINT]);
  });
  return table[rhs][tab];
}

// Grid of the forward launch: static mode covers n lanes; the persistent
// queue mode fills every CU to its occupancy limit (or takes the caller's
// grid) but never launches more lanes than trajectories.  `limit` is the
// grid before that last clip: the most workgroups the launch may hold.
void solve_shape(const gs_solve_args* a, int* grid, int* block, int64_t* limit = nullptr,
                 bool defer = true) {
  const int b = a->block > 0 ? a->block : 256;
  const int64_t need = (a->n + b - 1) / b;
  int64_t lim = need;
  if (a->schedule == GS_SCHED_STATIC) {
    *grid = (int)need;
  } else if (a->grid > 0) {
    lim = a->grid;
    *grid = (int)std::min<int64_t>(a->grid, need);
  } else {
    int per_cu = 0;
    const gs_host::Ops& o = ops(a->rhs, a->tableau);
    const void* fn = is_stiff(a) ? gs_host::stiff_solve_fn(a->rhs)
                     : (a->K > 0 && !defers_outputs(a, defer)) ? o.solve_fn_inloop
                                                                : o.solve_fn[a->K > 0][a->ckpt_every > 0];
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, b, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    lim = (int64_t)per_cu * num_cus();
    *grid = (int)std::min<int64_t>(lim, need);
  }
  *block = b;
  if (limit) *limit = lim;
}

// Split of a forward launch with `wide` trajectories on 16-lane groups.  The
// group workgroups (block / 16 groups each) and the single-lane workgroups
// draw from separate persistent queues.  Both together stay within `limit`
// (a persistent grid must be resident as a whole), except that each side
// that has trajectories gets at least one workgroup: the single lanes keep
// the workgroups they need, up to half of the limit, and the groups take
// the rest, as many as start every wide trajectory at once if that fits.
void wide_split(int64_t n, int64_t n_wide, int block, int64_t limit, int* wide_blocks,
                int* grid) {
  const int64_t per_block = block / gs::kGroup;
  const int64_t want_w = (n_wide + per_block - 1) / per_block;
  const int64_t need_s = (n - n_wide + block - 1) / block;
  const int64_t keep_s = std::min<int64_t>(need_s, std::max<int64_t>(limit / 2, 1));
  const int64_t w = std::min<int64_t>(want_w, std::max<int64_t>(limit - keep_s, 1));
  const int64_t single =
      need_s > 0 ? std::max<int64_t>(std::min<int64_t>(need_s, limit - w), 1) : 0;
  *wide_blocks = (int)w;
  *grid = (int)(w + single);
}

gs_status launch_solve_all(const gs_solve_args* a, bool defer = true) {
  hipStream_t s = static_cast<hipStream_t>(a->stream);
  const Params P = make_params(a, defer);
  Params P2 = P;
  hipLaunchKernelGGL(reset_queues_kernel, dim3(1), dim3(64), 0, s, P.counters, (long long)P.n_wide);
  if (a->order)
    hipLaunchKernelGGL(fill_status_kernel, dim3(fill_grid(P.n)), dim3(256), 0, s, P.status, P.n,
                       (int32_t)GS_TRAJ_NOT_RUN);
  int grid = 0, block = 0;
  int64_t limit = 0;
  solve_shape(a, &grid, &block, &limit, defer);
  if (is_stiff(a)) {
    gs_host::launch_stiff(a->rhs, P, grid, block, s);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
  }
  if (P.n_wide > 0) wide_split(P.n, P.n_wide, block, limit, &P2.wide_blocks, &grid);
  ops(a->rhs, a->tableau).solve(P2, grid, block, s);
  if (P.pending) ops(a->rhs, a->tableau).short_steps(P, s);
  return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

// Fixed scratch of gs_solve_noalloc: the work-queue counters of a solve
// without a tape (256 bytes used).  Each GPU the library runs on holds one
// copy until the process ends; host code reaches it only through the device
// address that hipGetSymbolAddress returns for the current device (the
// array's own name is a host-side stand-in).
constexpr size_t kStaticScratchBytes = 4096;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) on its first use.
gs_status static_scratch(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return GS_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) return GS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GS_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GS_OK;
}

// Workspace of gs_queue_order: keys, buckets, histogram, key range.
struct OrderLayout {
  size_t key, bucket, hist, range, total;
};
OrderLayout order_layout(int64_t n) {
  OrderLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align256(off + bytes);
    return at;
  };
  L.key = take((size_t)n * 8);
  L.bucket = take((size_t)n * 4);
  L.hist = take((size_t)gs::order::kBuckets * 4);
  L.range = take(16);
  L.total = off;
  return L;
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

gs_status gs_solve_noalloc(const gs_solve_args* a) {
  if (!a) return GS_ERR_INVALID;
  if (a->ckpt_every != 0) return GS_ERR_UNSUPPORTED;
  gs_solve_args c = *a;
  c.workspace = nullptr;
  c.workspace_bytes = kStaticScratchBytes;
  // Deferred outputs only where their records fit; a pair with a dense
  // polynomial then evaluates its outputs in the solve kernel instead.
  bool defer = true;
  if (c.rhs >= 0 && c.rhs < kNumRhs && c.n >= 0 && layout_of(&c).total > kStaticScratchBytes) {
    defer = false;
    if (layout_of(&c, false).total > kStaticScratchBytes) return GS_ERR_TOO_LARGE;
  }
  void* p = nullptr;
  const gs_status sp = static_scratch(&p);
  if (sp != GS_OK) return sp;
  c.workspace = p;
  const gs_status st = check_args(&c, defer);
  if (st != GS_OK || c.n == 0) return st;
  return launch_solve_all(&c, defer);
}

size_t gs_queue_order_workspace_bytes(int64_t n) {
  if (n < 0 || n > (int64_t)1 << 31) return 0;
  return order_layout(n).total;
}

gs_status gs_queue_order(const gs_solve_args* a, const double* cost, int64_t* order,
                         void* workspace, size_t workspace_bytes) {
  if (!a || !order) return GS_ERR_INVALID;
  if (a->rhs < 0 || a->rhs >= kNumRhs || a->tableau < 0 || a->tableau >= kNumTab || a->n < 0)
    return GS_ERR_INVALID;
  if (a->n > (int64_t)1 << 31) return GS_ERR_UNSUPPORTED;
  if (a->n == 0) return GS_OK;
  if (!cost) {
    if (!a->t0 || !a->t1 || !a->rtol) return GS_ERR_INVALID;
    if (a->t_stride != 0 && a->t_stride != 1) return GS_ERR_INVALID;
    if (a->tol_stride != 0 && a->tol_stride != 1) return GS_ERR_INVALID;
    if (a->rhs == GS_RHS_LOGHALO) {
      if (!a->y0 || !a->theta || a->d != rhs_dim(a->rhs) || a->p != rhs_np(a->rhs))
        return GS_ERR_INVALID;
      if (a->theta_stride != 0 && a->theta_stride != a->n) return GS_ERR_INVALID;
    }
  }
  const OrderLayout L = order_layout(a->n);
  if (!workspace || ((uintptr_t)workspace & 255) != 0 || workspace_bytes < L.total)
    return GS_ERR_WORKSPACE;
  char* ws = static_cast<char*>(workspace);
  gs::order::Ws w;
  w.key = reinterpret_cast<double*>(ws + L.key);
  w.bucket = reinterpret_cast<uint32_t*>(ws + L.bucket);
  w.hist = reinterpret_cast<uint32_t*>(ws + L.hist);
  w.range = reinterpret_cast<unsigned long long*>(ws + L.range);
  gs::order::CostIn c;
  std::memset(&c, 0, sizeof c);
  c.n = a->n;
  c.loghalo = (!cost && a->rhs == GS_RHS_LOGHALO) ? 1 : 0;
  c.inv_nu = 1.0 / tab_order(a->tableau);
  c.y0 = a->y0;
  c.theta = a->theta;
  c.theta_stride = a->theta_stride;
  c.t0 = a->t0;
  c.t1 = a->t1;
  c.t_stride = a->t_stride;
  c.rtol = a->rtol;
  c.tol_stride = a->tol_stride;
  c.cost = cost;
  hipStream_t s = static_cast<hipStream_t>(a->stream);
  const int grid = (int)((a->n + 255) / 256);
  hipLaunchKernelGGL(gs::order::clear_kernel, dim3(gs::order::kBuckets / 256), dim3(256), 0, s,
                     w);
  hipLaunchKernelGGL(gs::order::key_kernel, dim3(grid), dim3(256), 0, s, c, w);
  hipLaunchKernelGGL(gs::order::bucket_kernel, dim3(grid), dim3(256), 0, s, a->n, w);
  hipLaunchKernelGGL(gs::order::scan_kernel, dim3(1), dim3(gs::order::kScanThreads), 0, s, w);
  hipLaunchKernelGGL(gs::order::scatter_kernel, dim3(grid), dim3(256), 0, s, a->n, w, order);
  return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

gs_status gs_solve_vjp(const gs_solve_args* fwd, const gs_vjp_args* v) {
  gs_status st = check_args(fwd);
  if (st != GS_OK) return st;
  if (is_stiff(fwd)) return GS_ERR_UNSUPPORTED;
  if (!v || v->R < 1 || v->R > 8 || !v->y0bar || !v->thetabar) return GS_ERR_INVALID;
  if (v->ybar_out && fwd->K == 0) return GS_ERR_INVALID;
  if (fwd->ckpt_every <= 0) return GS_ERR_NO_TAPE;
  if (v->block != 0 && (v->block < 64 || v->block > 256 || v->block % 64 != 0))
    return GS_ERR_INVALID;
  if (v->wide < 0) return GS_ERR_INVALID;
  if (v->wide > 0 && (fwd->ckpt_every != 1 || fwd->K > 0)) return GS_ERR_UNSUPPORTED;
  if (fwd->n == 0) return GS_OK;
  const Layout L = layout_of(fwd);
  // The stage points of the step each lane reverses live in LDS, (s - 1) d
  // doubles per lane, when there are too many to keep in registers; a block
  // that would need more than the device allows per workgroup gets fewer
  // lanes.
  const size_t lds_lane = (size_t)ops(fwd->rhs, fwd->tableau).vjp_lds_lane[fwd->K > 0 ? 1 : 0];
  int block = v->block > 0 ? v->block : 256;
  while (block > 64 && lds_lane * block > max_lds_per_block()) block -= 64;
  if (lds_lane * block > max_lds_per_block()) return GS_ERR_UNSUPPORTED;
  hipStream_t s = static_cast<hipStream_t>(v->stream);
  Params P = make_params(fwd);
  P.n_wide = std::min<int64_t>(v->wide, fwd->n);  // the adjoint's own groups
  P.wide_blocks = 0;
  VjpParams V;
  std::memset(&V, 0, sizeof V);
  V.R = std::min(kVjpMaxR, (int)v->R);
  V.lds_bytes = (int32_t)(lds_lane * block);
  // Persistent grid: at most the lanes the workspace has scratch for, and no
  // more than fit on the device at once.
  int grid = (int)(L.adj_lanes / block);
  if (v->grid > 0) {
    grid = std::min(grid, v->grid);
  } else {
    int per_cu = 0;
    V.occupancy_out = &per_cu;
    ops(fwd->rhs, fwd->tableau).vjp(P, V, 0, block, s);
    V.occupancy_out = nullptr;
    if (per_cu > 0) grid = (int)std::min<int64_t>(grid, (int64_t)per_cu * num_cus());
  }
  if (grid < 1) return GS_ERR_INVALID;
  if (P.n_wide > 0) wide_split(P.n, P.n_wide, block, grid, &P.wide_blocks, &grid);
  V.R_total = v->R;
  V.ybar_out = v->ybar_out;
  V.ybar_final = v->ybar_final;
  V.y0bar = v->y0bar;
  V.thetabar = v->thetabar;
  V.scratch = reinterpret_cast<double*>(static_cast<char*>(fwd->workspace) + L.scratch_off);
  V.adj = reinterpret_cast<double*>(static_cast<char*>(fwd->workspace) + L.adj_off);
  hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, s, P.counters + 2, 1);
  if (fwd->order) {
    const int64_t my = (int64_t)v->R * fwd->d * fwd->n, mt = (int64_t)v->R * fwd->p * fwd->n;
    hipLaunchKernelGGL(fill_nan_kernel, dim3(fill_grid(my)), dim3(256), 0, s, v->y0bar, my);
    hipLaunchKernelGGL(fill_nan_kernel, dim3(fill_grid(mt)), dim3(256), 0, s, v->thetabar, mt);
  }
  for (int r0 = 0; r0 < v->R; r0 += kVjpMaxR) {
    V.r0 = r0;
    V.R = std::min(kVjpMaxR, v->R - r0);
    hipLaunchKernelGGL(reset_vjp_queues_kernel, dim3(1), dim3(64), 0, s, P.counters,
                       (long long)P.n_wide);
    ops(fwd->rhs, fwd->tableau).vjp(P, V, grid, block, s);
  }
  return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

namespace {
// The launches of a sensitivity solve whose arguments have been checked.
void sens_launches(const gs_solve_args* a, const gs_sens_args* sa) {
  hipStream_t s = static_cast<hipStream_t>(a->stream);
  const Params P = make_params(a);
  const int block = a->block > 0 ? a->block : 256;
  gs::SensParams S;
  std::memset(&S, 0, sizeof S);
  S.m_total = sa->M;
  S.S_final = sa->S_final;
  S.S_out = sa->S_out;
  if (a->order)
    hipLaunchKernelGGL(fill_status_kernel, dim3(fill_grid(P.n)), dim3(256), 0, s, P.status, P.n,
                       (int32_t)GS_TRAJ_NOT_RUN);
  // Two columns per launch; each launch integrates the solution again and
  // rewrites the same values.
  for (int m0 = 0; m0 < sa->M; m0 += 2) {
    const int mm = std::min(2, sa->M - m0);
    S.m0 = m0;
    for (int m = 0; m < 4; ++m) S.col[m] = m < mm ? sa->cols[m0 + m] : -1;
    const int64_t need = (a->n + block - 1) / block;
    int64_t limit = a->grid;
    if (a->grid <= 0) {
      int per_cu = 0;
      S.occupancy_out = &per_cu;
      ops(a->rhs, a->tableau).sens(P, S, mm, 0, block, s);
      S.occupancy_out = nullptr;
      limit = (int64_t)std::max(per_cu, 1) * num_cus();
    }
    // The head of the order on 16-lane groups, as in a plain solve.
    Params P2 = P;
    int grid = (int)std::min<int64_t>(limit, need);
    if (P.n_wide > 0) wide_split(P.n, P.n_wide, block, limit, &P2.wide_blocks, &grid);
    hipLaunchKernelGGL(reset_queues_kernel, dim3(1), dim3(64), 0, s, P.counters,
                       (long long)P.n_wide);
    ops(a->rhs, a->tableau).sens(P2, S, mm, grid, block, s);
  }
}

// Workspace of gs_de_profile: solver counters, device scalars (t0, t1, rtol,
// atol), theta [4][n], y0 [3][n], y_out [3][K][n], y_final [3][n],
// S_out [3][2][K][n], S_final [3][2][n], and three int32 [n] arrays.
struct DeLayout {
  size_t counters, scal, theta, y0, y_out, y_final, S_out, S_final, nacc, nrej, st;
  size_t W, tmp, total;  // spline only: weights and their scratch
};
DeLayout de_layout(const gs_de_profile_args* A) {
  DeLayout L;
  const size_t n = (size_t)A->n, K = (size_t)A->K;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align256(off + bytes);
    return at;
  };
  L.counters = take(kCounterBytes);
  L.scal = take(4 * 8);
  L.theta = take(4 * n * 8);
  L.y0 = take(3 * n * 8);
  L.y_out = take(3 * K * n * 8);
  L.y_final = take(3 * n * 8);
  L.S_out = take(3 * 2 * K * n * 8);
  L.S_final = take(3 * 2 * n * 8);
  L.nacc = take(n * 4);
  L.nrej = take(n * 4);
  L.st = take(n * 4);
  const size_t Kd = A->K_data > 0 ? (size_t)A->K_data : 0;
  L.W = take(Kd * K * 8);
  L.tmp = take(Kd ? 3 * K * K * 8 : 0);
  L.total = off;
  return L;
}

__global__ void de_setup_kernel(int64_t n, double* scal, double t0, double rtol, double atol,
                                double* y0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    scal[0] = t0;
    scal[1] = 0.0;
    scal[2] = rtol;
    scal[3] = atol;
  }
  if (i < 3 * n) y0[i] = 0.0;
}
}  // namespace

gs_status gs_solve_sens(const gs_solve_args* a, const gs_sens_args* sa) {
  gs_status st = check_args(a);
  if (st != GS_OK) return st;
  if (!sa || sa->M < 1 || sa->M > kSensMaxCols || !sa->cols || !sa->S_final) return GS_ERR_INVALID;
  if (a->K > 0 && !sa->S_out) return GS_ERR_INVALID;
  if (is_stiff(a) || a->ckpt_every > 0 || a->schedule != GS_SCHED_QUEUE)
    return GS_ERR_UNSUPPORTED;
  for (int m = 0; m < sa->M; ++m)
    if (sa->cols[m] < 0 || sa->cols[m] >= a->d + a->p) return GS_ERR_INVALID;
  if (a->n == 0) return GS_OK;
  sens_launches(a, sa);
  return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

size_t gs_de_profile_workspace_bytes(const gs_de_profile_args* A) {
  if (!A || A->n < 0 || A->K < 1 || A->K_data < 0) return 0;
  return de_layout(A).total;
}

gs_status gs_de_profile(const gs_de_profile_args* A) {
  if (!A || A->n < 0 || A->K < 1 || A->iters < 0 || A->newton < 0 || A->K_data < 0)
    return GS_ERR_INVALID;
  if (A->K_data > 0 && (A->K < 4 || !A->N_data)) return GS_ERR_INVALID;
  if (A->n > (int64_t)1 << 31) return GS_ERR_UNSUPPORTED;  // grid sizes are int
  if (A->tableau < 0 || A->tableau >= kNumExplicitTab || !(A->rtol > 0.0) || !(A->atol >= 0.0) ||
      !(A->N_start < 0.0) || !(A->mu >= 0.0) || !(A->trust_om > 0.0) || !(A->trust_h > 0.0))
    return GS_ERR_INVALID;
  if (A->n == 0) return GS_OK;
  if (!A->lambda || !A->omega_m || !A->h || !A->a0 || !A->N_nodes || !A->data || !A->sigma ||
      !A->chi2 || !A->chi2_prev || !A->decrement || !A->status)
    return GS_ERR_INVALID;
  if (!A->workspace || ((uintptr_t)A->workspace & 255) != 0 ||
      A->workspace_bytes < de_layout(A).total)
    return GS_ERR_WORKSPACE;
  const DeLayout L = de_layout(A);
  char* ws = static_cast<char*>(A->workspace);
  auto D = [&](size_t off) { return reinterpret_cast<double*>(ws + off); };
  auto I = [&](size_t off) { return reinterpret_cast<int32_t*>(ws + off); };
  const int64_t n = A->n;
  const int blk = 256;
  const int grd = (int)((n + blk - 1) / blk);
  const int grd3 = (int)((3 * n + blk - 1) / blk);
  hipStream_t s = static_cast<hipStream_t>(A->stream);
  hipLaunchKernelGGL(de_setup_kernel, dim3(grd3), dim3(blk), 0, s, n, D(L.scal), A->N_start,
                     A->rtol, A->atol, D(L.y0));
  hipLaunchKernelGGL(gs::de::init_kernel, dim3(grd), dim3(blk), 0, s, n, A->a0, A->lambda,
                     A->omega_m, A->omega_r, D(L.theta), A->status);
  // The ensemble solve of the quintessence system for the current theta.
  gs_solve_args a;
  gs_default_args(&a);
  a.rhs = GS_RHS_QUINT;
  a.tableau = A->tableau;
  a.n = n;
  a.d = 3;
  a.p = 4;
  a.y0 = D(L.y0);
  a.theta = D(L.theta);
  a.theta_stride = n;
  a.t0 = D(L.scal);
  a.t1 = D(L.scal) + 1;
  a.rtol = D(L.scal) + 2;
  a.atol = D(L.scal) + 3;
  a.t_out = A->N_nodes;
  a.y_out = D(L.y_out);
  a.y_final = D(L.y_final);
  a.n_accepted = I(L.nacc);
  a.n_rejected = I(L.nrej);
  a.status = I(L.st);
  a.workspace = ws + L.counters;
  a.workspace_bytes = kCounterBytes;
  a.stream = A->stream;
  const int32_t col_a0[1] = {3};          // d/da0
  const int32_t col_both[2] = {3, 5};     // d/da0, d/dOm
  gs_sens_args one{1, col_a0, D(L.S_final), nullptr};
  gs_sens_args both{2, col_both, D(L.S_final), D(L.S_out)};
  auto shoot = [&]() {
    a.K = 0;
    for (int j = 0; j < A->newton; ++j) {
      sens_launches(&a, &one);
      hipLaunchKernelGGL(gs::de::shoot_kernel, dim3(grd), dim3(blk), 0, s, n, D(L.theta),
                         D(L.y_final), D(L.S_final), I(L.st), A->status);
    }
    a.K = A->K;
  };
  gs::de::GnArgs g;
  g.n = n;
  g.K = A->K;
  g.N_nodes = A->N_nodes;
  g.y_out = D(L.y_out);
  g.y_final = D(L.y_final);
  g.S_out = D(L.S_out);
  g.S_final = D(L.S_final);
  g.data = A->data;
  g.sigma = A->sigma;
  g.Kd = A->K_data > 0 ? A->K_data : A->K;
  g.W = nullptr;
  if (A->K_data > 0) {
    hipLaunchKernelGGL(gs::de::spline_weights_kernel, dim3((A->K + 63) / 64), dim3(64), 0, s,
                       A->K, A->N_nodes, A->K_data, A->N_data, D(L.tmp), D(L.W));
    g.W = D(L.W);
  }
  g.status = I(L.st);
  g.mu = A->mu;
  g.trust_om = A->trust_om;
  g.trust_h = A->trust_h;
  g.theta = D(L.theta);
  g.h = A->h;
  g.chi2 = A->chi2;
  g.chi2_prev = A->chi2_prev;
  g.decrement = A->decrement;
  g.status_out = A->status;
  for (int it = 0; it < A->iters; ++it) {
    shoot();
    sens_launches(&a, &both);
    g.update = 1;
    g.dist = nullptr;
    hipLaunchKernelGGL(gs::de::gn_kernel, dim3(grd), dim3(blk), 0, s, g);
  }
  // chi2 and distances at the returned parameters, the amplitude flat there
  shoot();
  sens_launches(&a, &both);
  g.update = 0;
  g.dist = A->dist;
  hipLaunchKernelGGL(gs::de::gn_kernel, dim3(grd), dim3(blk), 0, s, g);
  hipLaunchKernelGGL(gs::de::finish_kernel, dim3(grd), dim3(blk), 0, s, n, D(L.theta), A->a0,
                     A->omega_m);
  return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

gs_status gs_dense_eval(const gs_solve_args* fwd, int32_t Q, const double* t_query,
                        double* y_query, void* stream) {
  const gs_status st = check_args(fwd);
  if (st != GS_OK) return st;
  if (is_stiff(fwd)) return GS_ERR_UNSUPPORTED;
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
  if (m > (int64_t)1 << 31) return GS_ERR_UNSUPPORTED;  // grid sizes are int
  if (m == 0) return GS_OK;
  if (!t || !y || !theta) return GS_ERR_INVALID;
  const bool want_vjp = kbar || ybar || thetabar;
  if (want_vjp && !(kbar && ybar && thetabar)) return GS_ERR_INVALID;
  const int block = 256;
  const int grid = (int)((m + block - 1) / block);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (rhs >= kNumExplicitRhs) {
    if (want_vjp) return GS_ERR_UNSUPPORTED;
    if (!f) return GS_ERR_INVALID;
    gs_host::launch_stiff_rhs(rhs, m, y, theta, f, s);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
  }
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
    case GS_ERR_TOO_LARGE: return "request exceeds the fixed static scratch of gs_solve_noalloc";
  }
  return "unknown status";
}

const char* gs_version(void) { return "0.2.0"; }

}  // extern "C"
