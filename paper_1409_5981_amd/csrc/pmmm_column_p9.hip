// Column-stage instantiations (pmmm_column.h) for order 9.
#include "pmmm_column.h"

namespace pmmm {

template hipError_t column_launch<9, float>(const FFTArgs &, hipStream_t);
template hipError_t column_launch<9, double>(const FFTArgs &, hipStream_t);

}  // namespace pmmm
