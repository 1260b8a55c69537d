// k_cov_np_60_64.hip -- the covariance build for padded bin counts 60, 64
// (split over several files to compile in parallel).
#include "k_cov_impl.h"

namespace fcx {

template hipError_t launch_cov_np<60>(const fc_grid *, const double *, const double *, int,
                                       uint32_t, const int16_t *, double *, uint4 *, uint4 *,
                                       uint4 *, uint4 *, unsigned long long *, hipStream_t);
template hipError_t launch_cov_np<64>(const fc_grid *, const double *, const double *, int,
                                       uint32_t, const int16_t *, double *, uint4 *, uint4 *,
                                       uint4 *, uint4 *, unsigned long long *, hipStream_t);

}  // namespace fcx
