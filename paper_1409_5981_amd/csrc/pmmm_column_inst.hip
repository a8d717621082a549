// Column-stage instantiations (pmmm_column.h) for one order and precision,
// PMMM_COLUMN_ORDER and PMMM_COLUMN_T, given by the build: the unit is
// compiled once per pair so that the orders build in parallel.
#include "pmmm_column.h"

#if !defined(PMMM_COLUMN_ORDER) || !defined(PMMM_COLUMN_T)
#error "compile with -DPMMM_COLUMN_ORDER=<0..PMMM_PMAX> -DPMMM_COLUMN_T=<float|double>"
#endif

namespace pmmm {

template hipError_t column_launch<PMMM_COLUMN_ORDER, PMMM_COLUMN_T>(const FFTArgs &, hipStream_t);

}  // namespace pmmm
