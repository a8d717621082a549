// Column-stage instantiations (pmmm_column.h) for order 10.
#include "pmmm_column.h"

namespace pmmm {

template hipError_t column_launch<10, float>(const FFTArgs &, hipStream_t);
template hipError_t column_launch<10, double>(const FFTArgs &, hipStream_t);

}  // namespace pmmm
