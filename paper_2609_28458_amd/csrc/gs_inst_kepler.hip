// Kernels of the Kepler right-hand side for every tableau.
#include "gs_inst.hpp"

namespace gs_host {
void ops_row_kepler(Ops* row) { fill_row<gs::Kepler>(row); }
}  // namespace gs_host
