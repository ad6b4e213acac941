// Kernels of the Quint right-hand side for every tableau.
#include "gs_inst.hpp"

namespace gs_host {
void ops_row_quint(Ops* row) { fill_row<gs::Quint>(row); }
}  // namespace gs_host
