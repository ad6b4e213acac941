// Kernel launchers of one (tableau, right-hand side) pair, and the tables
// that the C ABI dispatches through.  Each right-hand side's kernels are
// instantiated in a translation unit of their own (gs_inst_<rhs>.hip) so the
// library builds in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include "gs_kernels.hpp"

namespace gs_host {

struct Ops {
  // The forward kernel variants, [output nodes][tape], for the occupancy
  // query of the one that runs.
  const void* solve_fn[2][2];
  // The variant with outputs evaluated in the loop (pairs with a dense
  // polynomial, no pending array), or null.
  const void* solve_fn_inloop;
  void (*solve)(const gs::Params&, int grid, int block, hipStream_t);
  // grid <= 0: no launch; writes the blocks per CU of the variant that
  // would run to *V.occupancy_out.
  void (*vjp)(const gs::Params&, const gs::VjpParams&, int grid, int block, hipStream_t);
  void (*dense)(const gs::Params&, int32_t Q, const double*, double*, int grid, int block,
                hipStream_t);
  // Sensitivity solve with M (1 or 2) columns; grid <= 0 writes the blocks
  // per CU of the variant to *S.occupancy_out instead of launching.
  void (*sens)(const gs::Params&, const gs::SensParams&, int M, int grid, int block, hipStream_t);
  // The deferred shortened-step outputs of a plain solve (P.pending set).
  void (*short_steps)(const gs::Params&, hipStream_t);
  // Bytes of LDS per lane the adjoint uses for the stage points (0 when it
  // keeps them in registers), [output nodes].
  int vjp_lds_lane[2];
};

// Fill row[GS_DOPRI5], row[GS_TSIT5], row[GS_VERNER7] for one right-hand side.
void ops_row_harmonic(Ops* row);
void ops_row_kepler(Ops* row);
void ops_row_loghalo(Ops* row);
void ops_row_spinprec(Ops* row);
void ops_row_quint(Ops* row);

// Stiff path (gs_inst_stiff.hip): the Rodas4 kernel of a stiff right-hand
// side (GS_RHS_KIN3 / GS_RHS_KIN8), its function for the occupancy query,
// and the right-hand side evaluation.
const void* stiff_solve_fn(int rhs);
void launch_stiff(int rhs, const gs::Params& P, int grid, int block, hipStream_t s);
void launch_stiff_rhs(int rhs, int64_t m, const double* y, const double* theta, double* f,
                      hipStream_t s);
int stiff_dim(int rhs);
int stiff_np(int rhs);

}  // namespace gs_host
