// Fine-level kernel of the hierarchy (pmmm_hier_cell.h) for one order,
// PMMM_HIER_ORDER, given by the build: the unit is compiled once per order so
// that the orders build in parallel.
#include "pmmm_hier_cell.h"

#if !defined(PMMM_HIER_ORDER)
#error "compile with -DPMMM_HIER_ORDER=<0..PMMM_PMAX>"
#endif

namespace pmmm {

template hipError_t hier_cell_launch<PMMM_HIER_ORDER>(const HierArgs &, hipStream_t);

}  // namespace pmmm
