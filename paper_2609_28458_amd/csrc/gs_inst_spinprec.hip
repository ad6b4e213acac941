// Kernels of the SpinPrec right-hand side for every tableau.
#include "gs_inst.hpp"

namespace gs_host {
void ops_row_spinprec(Ops* row) { fill_row<gs::SpinPrec>(row); }
}  // namespace gs_host
