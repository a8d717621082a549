// Column-stage instantiations (pmmm_column.h) for orders 7, 8.
#include "pmmm_column.h"

namespace pmmm {

template hipError_t column_launch<7, float>(const FFTArgs &, hipStream_t);
template hipError_t column_launch<7, double>(const FFTArgs &, hipStream_t);
template hipError_t column_launch<8, float>(const FFTArgs &, hipStream_t);
template hipError_t column_launch<8, double>(const FFTArgs &, hipStream_t);

}  // namespace pmmm
