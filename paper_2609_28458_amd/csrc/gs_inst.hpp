// Instantiation of every kernel variant for one right-hand side (included by
// the gs_inst_<rhs>.hip translation units only).
#pragma once

#include "gradsolve.h"
#include "gs_ops.hpp"

namespace gs_host {

template <class TB, class F>
void launch_solve(const gs::Params& P, int grid, int block, hipStream_t s) {
  if constexpr (TB::POLY_DENSE) {
    // Outputs without a pending array (the no-allocation entry point, which
    // keeps no tape either) are evaluated in the loop.
    if (P.K > 0 && !P.pending) {
      hipLaunchKernelGGL((gs::solve_kernel<TB, F, true, false, true>), dim3(grid), dim3(block), 0,
                         s, P);
      return;
    }
  }
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

template <class TB, class F, bool NODES, bool STORE, bool WIDE = false>
void launch_vjp_r(const gs::Params& P, const gs::VjpParams& V, int grid, int block,
                  hipStream_t s) {
  const void* fn = reinterpret_cast<const void*>(&gs::vjp_kernel<TB, F, 1, NODES, STORE, WIDE>);
  if (grid <= 0) {
    // Occupancy query: blocks per CU of the variant that would launch.
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, V.lds_bytes) != hipSuccess)
      per_cu = 0;
    *V.occupancy_out = per_cu;
    return;
  }
  hipLaunchKernelGGL((gs::vjp_kernel<TB, F, 1, NODES, STORE, WIDE>), dim3(grid), dim3(block),
                     V.lds_bytes, s, P, V);
}

// The head of the order runs on 16-lane groups (P.n_wide > 0) only for a
// store-mode tape without output nodes; the host passes n_wide = 0 otherwise.
template <class TB, class F>
void launch_vjp(const gs::Params& P, const gs::VjpParams& V, int grid, int block, hipStream_t s) {
  if (P.K > 0) {
    if (P.store)
      launch_vjp_r<TB, F, true, true>(P, V, grid, block, s);
    else
      launch_vjp_r<TB, F, true, false>(P, V, grid, block, s);
  } else {
    if (P.store) {
      if (P.n_wide > 0)
        launch_vjp_r<TB, F, false, true, true>(P, V, grid, block, s);
      else
        launch_vjp_r<TB, F, false, true>(P, V, grid, block, s);
    } else {
      launch_vjp_r<TB, F, false, false>(P, V, grid, block, s);
    }
  }
}

template <class TB, class F>
void launch_dense(const gs::Params& P, int32_t Q, const double* tq, double* yq, int grid,
                  int block, hipStream_t s) {
  hipLaunchKernelGGL((gs::dense_kernel<TB, F>), dim3(grid), dim3(block), 0, s, P, Q, tq, yq);
}

template <class TB, class F, int M, bool NODES, bool WIDE>
void launch_sens_v(const gs::Params& P, const gs::SensParams& S, int grid, int block,
                   hipStream_t s) {
  const void* fn = reinterpret_cast<const void*>(&gs::sens_kernel<TB, F, M, NODES, WIDE>);
  if (grid <= 0) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, 0) != hipSuccess) per_cu = 0;
    *S.occupancy_out = per_cu;
    return;
  }
  hipLaunchKernelGGL((gs::sens_kernel<TB, F, M, NODES, WIDE>), dim3(grid), dim3(block), 0, s, P,
                     S);
}

template <class TB, class F, int M>
void launch_sens_m(const gs::Params& P, const gs::SensParams& S, int grid, int block,
                   hipStream_t s) {
  if (P.K > 0) {
    if (P.n_wide > 0)
      launch_sens_v<TB, F, M, true, true>(P, S, grid, block, s);
    else
      launch_sens_v<TB, F, M, true, false>(P, S, grid, block, s);
  } else {
    if (P.n_wide > 0)
      launch_sens_v<TB, F, M, false, true>(P, S, grid, block, s);
    else
      launch_sens_v<TB, F, M, false, false>(P, S, grid, block, s);
  }
}

template <class TB, class F>
void launch_sens(const gs::Params& P, const gs::SensParams& S, int M, int grid, int block,
                 hipStream_t s) {
  if (M >= 2)
    launch_sens_m<TB, F, 2>(P, S, grid, block, s);
  else
    launch_sens_m<TB, F, 1>(P, S, grid, block, s);
}

template <class TB, class F>
void launch_short_steps(const gs::Params& P, hipStream_t s) {
  const int64_t m = (int64_t)P.K * P.n;
  hipLaunchKernelGGL((gs::short_step_kernel<TB, F>), dim3((unsigned)((m + 255) / 256)), dim3(256), 0,
                     s, P);
}

template <class TB, class F>
Ops make_ops() {
  const void* inloop = nullptr;
  if constexpr (TB::POLY_DENSE)
    inloop = reinterpret_cast<const void*>(&gs::solve_kernel<TB, F, true, false, true>);
  return Ops{{{reinterpret_cast<const void*>(&gs::solve_kernel<TB, F, false, false>),
               reinterpret_cast<const void*>(&gs::solve_kernel<TB, F, false, true>)},
              {reinterpret_cast<const void*>(&gs::solve_kernel<TB, F, true, false>),
               reinterpret_cast<const void*>(&gs::solve_kernel<TB, F, true, true>)}},
             inloop,
             &launch_solve<TB, F>, &launch_vjp<TB, F>, &launch_dense<TB, F>, &launch_sens<TB, F>,
             &launch_short_steps<TB, F>,
             {gs::vjp_stages_in_lds<TB, F, false>() ? (TB::S - 1) * F::D * 8 : 0,
              gs::vjp_stages_in_lds<TB, F, true>() ? (TB::S - 1) * F::D * 8 : 0}};
}

template <class F>
void fill_row(Ops* row) {
  row[GS_DOPRI5] = make_ops<gs::Dopri5, F>();
  row[GS_TSIT5] = make_ops<gs::Tsit5, F>();
  row[GS_VERNER7] = make_ops<gs::Verner7, F>();
}

}  // namespace gs_host
