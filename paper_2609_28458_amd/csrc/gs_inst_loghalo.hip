// Kernels of the LogHalo right-hand side for every tableau.
#include "gs_inst.hpp"

namespace gs_host {
void ops_row_loghalo(Ops* row) { fill_row<gs::LogHalo>(row); }
}  // namespace gs_host
