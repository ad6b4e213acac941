// Kernels of the stiff path: Rodas4 on the stiff right-hand sides (the two
// kinetics networks, Robertson's reaction and HIRES).
#include "gradsolve.h"
#include "gs_ops.hpp"
#include "gs_stiff.hpp"

namespace gs_host {

namespace {
// Calls fn with a value of the stiff right-hand side's type.
template <class Fn>
void with_stiff(int rhs, Fn&& fn) {
  switch (rhs) {
    case GS_RHS_KIN3: fn(gs::Kin3{}); break;
    case GS_RHS_KIN8: fn(gs::Kin8{}); break;
    case GS_RHS_ROBER: fn(gs::Rober{}); break;
    default: fn(gs::Hires{}); break;
  }
}
}  // namespace

const void* stiff_solve_fn(int rhs) {
  const void* out = nullptr;
  with_stiff(rhs, [&](auto F) {
    out = reinterpret_cast<const void*>(&gs::stiff_kernel<decltype(F)>);
  });
  return out;
}

void launch_stiff(int rhs, const gs::Params& P, int grid, int block, hipStream_t s) {
  with_stiff(rhs, [&](auto F) {
    hipLaunchKernelGGL(gs::stiff_kernel<decltype(F)>, dim3(grid), dim3(block), 0, s, P);
  });
}

void launch_stiff_rhs(int rhs, int64_t m, const double* y, const double* theta, double* f,
                      hipStream_t s) {
  const int block = 256;
  const int grid = (int)((m + block - 1) / block);
  with_stiff(rhs, [&](auto F) {
    hipLaunchKernelGGL(gs::stiff_rhs_kernel<decltype(F)>, dim3(grid), dim3(block), 0, s, m, y,
                       theta, f);
  });
}

int stiff_dim(int rhs) {
  int d = 0;
  with_stiff(rhs, [&](auto F) { d = decltype(F)::D; });
  return d;
}
int stiff_np(int rhs) {
  int p = 0;
  with_stiff(rhs, [&](auto F) { p = decltype(F)::P; });
  return p;
}

}  // namespace gs_host
