// Kernels of the Harmonic right-hand side for every tableau.
#include "gs_inst.hpp"

namespace gs_host {
void ops_row_harmonic(Ops* row) { fill_row<gs::Harmonic>(row); }
}  // namespace gs_host
