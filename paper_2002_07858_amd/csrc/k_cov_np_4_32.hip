// k_cov_np_4_32.hip -- the covariance build for padded bin counts 4, 8, 12, 16, 20, 24, 28, 32
// (split over several files to compile in parallel).
#include "k_cov_impl.h"

namespace fcx {

template hipError_t launch_cov_np<4>(const fc_grid *, const double *, const double *, int,
                                       uint32_t, const int16_t *, double *, uint4 *, uint4 *,
                                       uint4 *, uint4 *, unsigned long long *, hipStream_t);
template hipError_t launch_cov_np<8>(const fc_grid *, const double *, const double *, int,
                                       uint32_t, const int16_t *, double *, uint4 *, uint4 *,
                                       uint4 *, uint4 *, unsigned long long *, hipStream_t);
template hipError_t launch_cov_np<12>(const fc_grid *, const double *, const double *, int,
                                       uint32_t, const int16_t *, double *, uint4 *, uint4 *,
                                       uint4 *, uint4 *, unsigned long long *, hipStream_t);
template hipError_t launch_cov_np<16>(const fc_grid *, const double *, const double *, int,
                                       uint32_t, const int16_t *, double *, uint4 *, uint4 *,
                                       uint4 *, uint4 *, unsigned long long *, hipStream_t);
template hipError_t launch_cov_np<20>(const fc_grid *, const double *, const double *, int,
                                       uint32_t, const int16_t *, double *, uint4 *, uint4 *,
                                       uint4 *, uint4 *, unsigned long long *, hipStream_t);
template hipError_t launch_cov_np<24>(const fc_grid *, const double *, const double *, int,
                                       uint32_t, const int16_t *, double *, uint4 *, uint4 *,
                                       uint4 *, uint4 *, unsigned long long *, hipStream_t);
template hipError_t launch_cov_np<28>(const fc_grid *, const double *, const double *, int,
                                       uint32_t, const int16_t *, double *, uint4 *, uint4 *,
                                       uint4 *, uint4 *, unsigned long long *, hipStream_t);
template hipError_t launch_cov_np<32>(const fc_grid *, const double *, const double *, int,
                                       uint32_t, const int16_t *, double *, uint4 *, uint4 *,
                                       uint4 *, uint4 *, unsigned long long *, hipStream_t);

}  // namespace fcx
