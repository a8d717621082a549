// Column-stage instantiations (pmmm_column.h) for orders 0, 1, 2, 3, 4.
#include "pmmm_column.h"

namespace pmmm {

template hipError_t column_launch<0, float>(const FFTArgs &, hipStream_t);
template hipError_t column_launch<0, double>(const FFTArgs &, hipStream_t);
template hipError_t column_launch<1, float>(const FFTArgs &, hipStream_t);
template hipError_t column_launch<1, double>(const FFTArgs &, hipStream_t);
template hipError_t column_launch<2, float>(const FFTArgs &, hipStream_t);
template hipError_t column_launch<2, double>(const FFTArgs &, hipStream_t);
template hipError_t column_launch<3, float>(const FFTArgs &, hipStream_t);
template hipError_t column_launch<3, double>(const FFTArgs &, hipStream_t);
template hipError_t column_launch<4, float>(const FFTArgs &, hipStream_t);
template hipError_t column_launch<4, double>(const FFTArgs &, hipStream_t);

}  // namespace pmmm
