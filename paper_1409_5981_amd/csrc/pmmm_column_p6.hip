// Column-stage instantiations (pmmm_column.h) for orders 6.
#include "pmmm_column.h"

namespace pmmm {

template hipError_t column_launch<6, float>(const FFTArgs &, hipStream_t);
template hipError_t column_launch<6, double>(const FFTArgs &, hipStream_t);

}  // namespace pmmm
