// Kernels of the stiff path: Rodas4 on the stiff kinetics right-hand sides.
#include "gradsolve.h"
#include "gs_ops.hpp"
#include "gs_stiff.hpp"

namespace gs_host {

const void* stiff_solve_fn(int rhs) {
  if (rhs == GS_RHS_KIN3) return reinterpret_cast<const void*>(&gs::stiff_kernel<gs::Kin3>);
  return reinterpret_cast<const void*>(&gs::stiff_kernel<gs::Kin8>);
}

void launch_stiff(int rhs, const gs::Params& P, int grid, int block, hipStream_t s) {
  if (rhs == GS_RHS_KIN3)
    hipLaunchKernelGGL(gs::stiff_kernel<gs::Kin3>, dim3(grid), dim3(block), 0, s, P);
  else
    hipLaunchKernelGGL(gs::stiff_kernel<gs::Kin8>, dim3(grid), dim3(block), 0, s, P);
}

void launch_stiff_rhs(int rhs, int64_t m, const double* y, const double* theta, double* f,
                      hipStream_t s) {
  const int block = 256;
  const int grid = (int)((m + block - 1) / block);
  if (rhs == GS_RHS_KIN3)
    hipLaunchKernelGGL(gs::stiff_rhs_kernel<gs::Kin3>, dim3(grid), dim3(block), 0, s, m, y,
                       theta, f);
  else
    hipLaunchKernelGGL(gs::stiff_rhs_kernel<gs::Kin8>, dim3(grid), dim3(block), 0, s, m, y,
                       theta, f);
}

int stiff_dim(int rhs) { return rhs == GS_RHS_KIN3 ? gs::Kin3::D : gs::Kin8::D; }
int stiff_np(int rhs) { return rhs == GS_RHS_KIN3 ? gs::Kin3::P : gs::Kin8::P; }

}  // namespace gs_host
