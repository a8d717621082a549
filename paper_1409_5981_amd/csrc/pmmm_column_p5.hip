// Column-stage instantiations (pmmm_column.h) for orders 5.
#include "pmmm_column.h"

namespace pmmm {

template hipError_t column_launch<5, float>(const FFTArgs &, hipStream_t);
template hipError_t column_launch<5, double>(const FFTArgs &, hipStream_t);

}  // namespace pmmm
