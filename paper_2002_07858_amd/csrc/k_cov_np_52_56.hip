// k_cov_np_52_56.hip -- the covariance build for padded bin counts 52, 56
// (split over several files to compile in parallel).
#include "k_cov_impl.h"

namespace fcx {

template hipError_t launch_cov_np<52>(const fc_grid *, const double *, const double *, int,
                                       uint32_t, const int16_t *, double *, uint4 *, uint4 *,
                                       uint4 *, uint4 *, unsigned long long *, hipStream_t);
template hipError_t launch_cov_np<56>(const fc_grid *, const double *, const double *, int,
                                       uint32_t, const int16_t *, double *, uint4 *, uint4 *,
                                       uint4 *, uint4 *, unsigned long long *, hipStream_t);

}  // namespace fcx
